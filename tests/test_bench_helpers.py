"""Host-side pieces of bench.py: the algorithmic byte count of the SpMV-step kernel and the rule that
reports counter traffic only while the SpMV source is the one the counters were taken on."""
import hashlib
import os

import bench


def test_spmv_step_bytes_by_hand():
    # CSR: 10 entries, 4 rows: matrix 10 * (8 + 4) + 4 * 5 = 140 B.  n = 2 (S column in the SpMV
    # epilogue): input + n - i columns of Q + output, i = 0, 1: 4 and 3, mean 3.5 vectors of 32 B
    assert bench.spmv_step_bytes(10, 4, 4, 2, 8) == 140 + 3.5 * 32
    # n = 8 real: the S column comes from the alpha pass, the step reads one column of Q: 3 vectors
    assert bench.spmv_step_bytes(10, 4, 4, 8, 8) == 140 + 3 * 32
    # transpose-free n = 8: 2 + 8 - i, i = 0..7: 10 + 9 + ... + 3 = 52, mean 6.5
    assert bench.spmv_step_bytes(10, 4, 4, 8, 8, transpose_free=True) == 140 + 6.5 * 32
    # complex values double the value bytes; n = 8 keeps the alpha-pass S column (17 x 16 B <= 288 B),
    # n = 16 does not (33 x 16 B): 3 + 4 + ... + 18 = 168 over 16 launches
    assert bench.spmv_step_bytes(10, 4, 4, 8, 16) == 10 * 20 + 20 + 3 * 64
    assert bench.spmv_step_bytes(10, 4, 4, 16, 16) == 10 * 20 + 20 + 10.5 * 64
    assert bench.spmv_step_bytes(10, 4, 4, 20, 8) == 140 + (sum(2 + 20 - i for i in range(20)) / 20) * 32
    # BSR3: 2 blocks, 2 block rows (N = 6), n = 1: 2 * (72 + 4) + 4 * 3 = 164 B; 3 vectors of 48 B
    assert bench.spmv_step_bytes(2, 2, 6, 1, 8, bsr=True) == 164 + 3 * 48


def _tree(tmp_path, src_text, recorded_hash, traffic=12345):
    csrc = tmp_path / "paper_1106_3678_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "mlb_spmv.hpp").write_text(src_text)
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "spmv_step_w.md").write_text(f"# x\n\ntraffic_bytes_per_launch: {traffic}\n"
                                         f"kernel_source_sha256: {recorded_hash}\n")
    return str(tmp_path)


def test_traffic_reported_only_for_the_measured_source(tmp_path):
    text = "// spmv kernels\n"
    good = hashlib.sha256(text.encode()).hexdigest()
    root = _tree(tmp_path / "a", text, good)
    assert bench.measured_traffic("w", root=root) == 12345
    root = _tree(tmp_path / "b", text + "// edited\n", good)
    assert bench.measured_traffic("w", root=root) is None
    assert bench.measured_traffic("missing", root=root) is None


def test_committed_profiles_parse():
    """Every committed SpMV-step summary carries a traffic figure and a source hash."""
    prof = os.path.join(bench.ROOT, "profiles")
    names = [f for f in os.listdir(prof) if f.startswith("spmv_step_") and f.endswith(".md")]
    assert names
    for f in names:
        text = open(os.path.join(prof, f)).read()
        assert "traffic_bytes_per_launch:" in text and "kernel_source_sha256:" in text
        assert "rocprofv3 --kernel-trace --stats" in text and "rocprofv3 --pmc FETCH_SIZE" in text


def test_cpu_baseline_sample_is_bounded():
    """The oracle baseline runs a bounded sample: the whole solve when it is short (counted as whole only
    when the oracle converged), else about target_s of CPU time scaled to the GPU's iteration count, and
    never beyond an explicit cap; both the single-core and the all-core runs are reported."""
    import workloads

    p = workloads.config1(n=4)
    whole = bench.cpu_baseline(p, 69, 0, 1e6, target_s=30.0, add_mib=8)
    assert whole["kind"] == "oracle" and "whole solve" in whole["sample"] and whole["whole"]
    assert whole["oracle_flag"] == 0 and whole["oracle_iter"] == 69
    assert whole["single_core"]["whole"] and whole["single_core"]["oracle_iter"] == 69
    assert whole["cores"] >= 1 and whole["host"]["threads_used"] == whole["cores"]
    assert whole["host"]["add_bandwidth_gbs"] > 0 and 0 < whole["bandwidth_frac"]
    capped = bench.cpu_baseline(p, 69, 10, 1e6, target_s=30.0, add_mib=8)
    assert "first 10 iterations" in capped["sample"] and not capped["whole"] and capped["oracle_flag"] == 1
    assert capped["value"] > 0
    short = bench.cpu_baseline(p, 69, 0, 1e6, target_s=1e-6, add_mib=8)
    assert "first 5 iterations" in short["sample"]


def test_vector_passes_by_hand():
    """x updates deferred to the omega pass (no iterate record).  n = 2: inner step i = 1 moves
    (3 + 1) + (2 + 2 + 1) + (2 + 1) + (2 + 1) = 15 vectors, the cycle end 3 + 2 + 9 + 6 + 4 = 24;
    39 per cycle of 2 iterations.  n = 1 (BiCGStab): 3 + 2 + 7 + 4 + 3 = 19 per iteration.  n = 4:
    inner steps 25 - 2i (23 + 21 + 19), cycle end 3 + 2 + 13 + 10 + 6 = 34; 97 per cycle.  n = 8 (S
    column from the alpha pass, every SpMV step 3 vectors): inner steps (11 - i) + (18 - i) + (2 + i) + 3
    = 34 - i, i = 1..7: 210; cycle end 3 + 2 + 21 + 18 + 3 = 47; 257 per cycle, n(n - 1)/2 = 28 fewer
    than with the S column in the SpMV epilogue."""
    assert bench.vector_passes_per_iter(2) == 39 / 2
    assert bench.vector_passes_per_iter(1) == 19
    assert bench.vector_passes_per_iter(4) == 97 / 4
    assert bench.vector_passes_per_iter(8) == 257 / 8
    assert bench.vector_passes_per_iter(8, sv=16) == 257 / 8
    assert bench.vector_passes_per_iter(16, sv=16) * 16 - bench.vector_passes_per_iter(16) * 16 == 16 * 15 / 2
    # transpose-free, n = 2: (3 + 1) + (2 + 2) + (2 + 1) + (4 + 2 + 1) = 18 per inner step
    assert bench.vector_passes_per_iter(2, transpose_free=True) == (18 + 24) / 2


def test_spmv_step_bytes_literal_order():
    """The literal order reduces one column of Q per SpMV step: input, one column, output."""
    nnz, N, n, sv = 7000, 1000, 8, 8
    mat = nnz * (sv + 4) + 4 * (N + 1)
    assert bench.spmv_step_bytes(nnz, N, N, n, sv, literal=True) == mat + 3 * N * sv
    assert bench.spmv_step_bytes(nnz, N, N, n, sv, literal=True, transpose_free=True) == mat + 3 * N * sv
    assert bench.spmv_step_bytes(nnz, N, N, n, sv, transpose_free=True) > mat + 3 * N * sv
