"""The C ABI: the library loads, exports every entry point the header declares, and rejects bad
arguments before touching a GPU (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mlbicgstab.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mlb(?:icgstab)?_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def binding():
    from paper_1106_3678_amd import lib_built

    if not lib_built():
        pytest.fail("libmlbicgstab.so is not built (run __graft_entry__.build())")
    from paper_1106_3678_amd import binding as b
    return b


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("mlbicgstab_create", "mlbicgstab_solve", "mlbicgstab_destroy", "mlbicgstab_workspace_size",
              "mlbicgstab_last_error", "mlbicgstab_time_kernel", "mlbicgstab_solve_batch", "mlb_server_create",
              "mlb_sequence_next_n", "mlb_sequence_create", "mlb_sequence_solve", "mlb_sequence_destroy",
              "mlb_server_submit",
              "mlb_server_poll", "mlb_server_wait", "mlb_server_stats", "mlb_server_destroy"):
        assert f in names


def test_library_exports_every_declared_symbol(binding):
    lib = ctypes.CDLL(binding.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def _desc(binding, **kw):
    d = dict(format=binding.MLB_CSR, dtype=binding.MLB_R64, nrows=10, nnz=10, row_ptr=1, col_idx=1, values=1)
    d.update(kw)
    return binding.mlb_matrix(**d)


def _opt(binding, **kw):
    o = dict(n=4, tol=1e-10, maxit=100, kappa=0.0, precision=0, inner_tol=0.0, max_outer=0, record_iterates=0,
             iterates=None, precond=0, transpose_free=0, order=0, max_restarts=0)
    o.update(kw)
    return binding.mlb_options(**o)


@pytest.mark.parametrize("bad", [
    dict(m=dict(format=7)), dict(m=dict(dtype=9)), dict(m=dict(nrows=0)), dict(m=dict(nrows=10, format=1)),
    dict(m=dict(nnz=-1)), dict(m=dict(row_ptr=None)),
    dict(m=dict(nrows=2 ** 31 - 2 ** 20 + 1)), dict(m=dict(nrows=2 ** 31 - 1)),
    dict(m=dict(nnz=2 ** 31 - 2 ** 20 + 1)), dict(m=dict(nrows=3 * 2 ** 30, format=1)),
    dict(o=dict(n=0)), dict(o=dict(tol=0.0)), dict(o=dict(tol=float("nan"))), dict(o=dict(maxit=0)),
    dict(o=dict(kappa=-1.0)), dict(o=dict(precision=5)), dict(o=dict(record_iterates=3)),
    dict(o=dict(precond=7)), dict(o=dict(transpose_free=2)), dict(o=dict(order=5)),
    dict(o=dict(max_restarts=-1)), dict(o=dict(max_restarts=101)),
])
def test_create_rejects_bad_arguments(binding, bad):
    A = _desc(binding, **bad.get("m", {}))
    o = _opt(binding, **bad.get("o", {}))
    h = binding.mlb_handle()
    rc = binding.raw_call("mlbicgstab_create", ctypes.byref(A), ctypes.byref(o), None, ctypes.byref(h))
    assert rc == binding.MLB_EINVAL
    assert h.value is None
    assert binding.mlbicgstab_last_error() != ""


def test_literal_order_with_transpose_free_is_unsupported(binding):
    A = _desc(binding)
    o = _opt(binding, order=binding.MLB_ORDER_LITERAL, transpose_free=1)
    h = binding.mlb_handle()
    rc = binding.raw_call("mlbicgstab_create", ctypes.byref(A), ctypes.byref(o), None, ctypes.byref(h))
    assert rc == binding.MLB_EUNSUPPORTED and h.value is None


def test_restarts_with_refinement_are_unsupported(binding):
    A = _desc(binding)
    o = _opt(binding, precision=binding.MLB_PREC_FP32_IR, max_restarts=1)
    h = binding.mlb_handle()
    rc = binding.raw_call("mlbicgstab_create", ctypes.byref(A), ctypes.byref(o), None, ctypes.byref(h))
    assert rc == binding.MLB_EUNSUPPORTED and h.value is None


def test_n_above_max_is_unsupported(binding):
    A = _desc(binding)
    o = _opt(binding, n=33)
    h = binding.mlb_handle()
    rc = binding.raw_call("mlbicgstab_create", ctypes.byref(A), ctypes.byref(o), None, ctypes.byref(h))
    assert rc == binding.MLB_EUNSUPPORTED


def test_null_handle_paths(binding):
    res = binding.mlb_result()
    assert binding.raw_call("mlbicgstab_solve", None, None, None, None, ctypes.c_int64(1),
                            ctypes.byref(res)) == binding.MLB_EINVAL
    assert binding.raw_call("mlbicgstab_destroy", None) == 0
    ms = ctypes.c_double()
    assert binding.raw_call("mlbicgstab_time_kernel", None, 0, 1, ctypes.byref(ms)) == binding.MLB_EINVAL
    assert binding.raw_call("mlbicgstab_matvec", None, binding.MLB_OP_A, None, None) == binding.MLB_EINVAL
    # batched solves: NULL arrays and an empty batch are refused before anything runs
    assert binding.raw_call("mlbicgstab_solve_batch", None, 1, None, None, None, None, None) == binding.MLB_EINVAL
    hs = (binding.mlb_handle * 1)()
    ptrs = (ctypes.c_void_p * 1)()
    lds = (ctypes.c_int64 * 1)(1)
    assert binding.raw_call("mlbicgstab_solve_batch", hs, 0, ptrs, ptrs, ptrs, lds, None) == binding.MLB_EINVAL
    assert binding.raw_call("mlbicgstab_solve_batch", hs, 1, ptrs, ptrs, ptrs, lds, None) == binding.MLB_EINVAL


def test_workspace_size_model(binding):
    """(4n+4)N-type footprint: grows linearly in n and N (Table 4.3 storage)."""
    s1 = binding.mlbicgstab_workspace_size(_desc(binding, nrows=30000, nnz=150000), _opt(binding, n=4))
    s2 = binding.mlbicgstab_workspace_size(_desc(binding, nrows=30000, nnz=150000), _opt(binding, n=8))
    s3 = binding.mlbicgstab_workspace_size(_desc(binding, nrows=60000, nnz=300000), _opt(binding, n=4))
    assert s2 > s1 and s3 > 1.9 * s1
    # 3 vectors (G, W, F) per extra shadow vector, 8 bytes each
    assert abs((s2 - s1) - 4 * 3 * 30000 * 8) < 1024


@pytest.mark.parametrize("n", [1, 4, 16])
@pytest.mark.parametrize("dtype,fmt", [(0, 0), (1, 0), (0, 1)])
def test_workspace_size_transpose_free(binding, n, dtype, fmt):
    """Without A^H the footprint drops by A^H (row pointers, indices, values) and by the
    n - 1 columns of F ((3n + 5) N instead of (4n + 4) N, Tables 4.2 and 4.3)."""
    N, nnz = 30000, 150000 // (9 if fmt else 1)
    sv = 16 if dtype else 8
    bs = 9 if fmt else 1
    nbr = N // 3 if fmt else N
    desc = _desc(binding, nrows=N, nnz=nnz, dtype=dtype, format=fmt)
    full = binding.mlbicgstab_workspace_size(desc, _opt(binding, n=n))
    tf = binding.mlbicgstab_workspace_size(desc, _opt(binding, n=n, transpose_free=1))
    ah = (nbr + 1) * 4 + nnz * 4 + nnz * bs * sv
    f = max(n - 1, 1) * N * sv
    assert full - tf == ah + f
    # the fp32 refinement mode also drops the fp32 copy of A^H's values and the fp32 F
    full32 = binding.mlbicgstab_workspace_size(desc, _opt(binding, n=n, precision=1))
    tf32 = binding.mlbicgstab_workspace_size(desc, _opt(binding, n=n, precision=1, transpose_free=1))
    assert full32 - tf32 == ah + f + nnz * bs * sv // 2 + f // 2


def test_server_rejects_bad_options(binding):
    h = binding.mlb_server_handle()
    for budget, inflight, small, order, wait in [(0, 4, 0, 0, 0.0), (1 << 30, 0, 0, 0, 0.0), (1 << 30, 65, 0, 0, 0.0),
                                                 (1 << 30, 4, -2, 0, 0.0), (1 << 30, 4, (1 << 18) + 1, 0, 0.0),
                                                 (1 << 30, 4, 0, 2, 0.0), (1 << 30, 4, 0, -1, 0.0),
                                                 (1 << 30, 4, 0, 1, -1.0), (1 << 30, 4, 0, 1, float("nan")),
                                                 (1 << 30, 4, 0, 1, float("inf"))]:
        o = binding.mlb_server_options(budget, inflight, small, order, wait)
        assert binding.raw_call("mlb_server_create", ctypes.byref(o), ctypes.byref(h)) == binding.MLB_EINVAL
        assert h.value is None
    assert binding.raw_call("mlb_server_destroy", None) == 0


def test_sequence_rule(binding):
    """Section 5.2: with t1, t2 the times of the previous and the current system, the next system uses
    n + step if t1 > t2 and n - step otherwise (kept within [n_min, n_max]); no previous time keeps n."""
    f = binding.mlb_sequence_next_n
    assert f(4, 10.0, 8.0, 2, 1, 16) == 6       # faster than before: n + step
    assert f(4, 8.0, 10.0, 2, 1, 16) == 2       # slower: n - step
    assert f(4, 9.0, 9.0, 2, 1, 16) == 2        # not faster: n - step
    assert f(15, 10.0, 8.0, 2, 1, 16) == 16     # clamped at n_max
    assert f(2, 8.0, 10.0, 4, 2, 16) == 2       # clamped at n_min
    assert f(4, -1.0, 8.0, 2, 1, 16) == 4       # first system: no previous time
    assert f(4, 10.0, 8.0, 0, 1, 16) == 4       # step 0 fixes n
    for bad in [(4, 1.0, 2.0, -1, 1, 16), (4, 1.0, 2.0, 1, 0, 16), (4, 1.0, 2.0, 1, 5, 4), (4, 1.0, 2.0, 1, 1, 33),
                (17, 1.0, 2.0, 1, 1, 16)]:
        assert f(*bad) == binding.MLB_EINVAL


def test_sequence_create_rejects_bad_bounds(binding):
    A = _desc(binding)
    h = binding.mlb_sequence_handle()
    for n, lo, hi, step in [(4, 5, 8, 1), (4, 1, 3, 1), (4, 0, 8, 1), (4, 1, 8, -1)]:
        o = _opt(binding, n=n)
        rc = binding.raw_call("mlb_sequence_create", ctypes.byref(A), ctypes.byref(o), lo, hi, step, None,
                              ctypes.byref(h))
        assert rc == binding.MLB_EINVAL and h.value is None
    o = _opt(binding, n=4)
    assert binding.raw_call("mlb_sequence_create", ctypes.byref(A), ctypes.byref(o), 1, 40, 1, None,
                            ctypes.byref(h)) == binding.MLB_EUNSUPPORTED
    res = binding.mlb_result()
    assert binding.raw_call("mlb_sequence_solve", None, None, None, None, ctypes.c_int64(1), ctypes.byref(res),
                            None) == binding.MLB_EINVAL
    assert binding.raw_call("mlb_sequence_destroy", None) == 0


STRUCTS = ("mlb_matrix", "mlb_options", "mlb_result", "mlb_server_options", "mlb_request_timing",
           "mlb_server_stats_t")


def test_binding_structs_and_constants_match_the_header(binding, tmp_path):
    """The ctypes structs have the header's sizes and field offsets, and every enum constant of the
    header has the binding's value: a C program compiled with gcc against include/mlbicgstab.h
    prints sizeof and offsetof of each binding field (a field the header lacks fails to compile)."""
    import shutil
    import subprocess

    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "%s"' % HEADER, "int main(void) {"]
    for sname in STRUCTS:
        st = getattr(binding, sname)
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (sname, sname))
        for fname, _ in st._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (sname, fname, sname, fname))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-std=c11", "-o", str(exe), str(src)], check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                  text=True).stdout.splitlines())
    for sname in STRUCTS:
        st = getattr(binding, sname)
        assert int(out[sname]) == ctypes.sizeof(st), sname
        for fname, _ in st._fields_:
            assert int(out[f"{sname}.{fname}"]) == getattr(st, fname).offset, (sname, fname)
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    consts = {}
    for body in re.findall(r"enum\s*\{(.*?)\}", text, flags=re.S):
        for name, val in re.findall(r"(MLB_\w+)\s*=\s*(-?\d+)", body):
            consts[name] = int(val)
    assert len(consts) >= 20
    for name, val in consts.items():
        assert getattr(binding, name) == val, name
