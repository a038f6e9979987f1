"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import numpy as np

import pytest

from paper_2004_02583_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tucker_als.h")

FAKE = ctypes.c_void_p(0x100000)  # never dereferenced: validation comes first


@pytest.fixture(scope="module")
def lib():
    return L.load_library()


def header_symbols():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^TK_API\s+[\w\s\*]*?\b(\w+)\s*\(", src, re.M)))


def test_header_symbols_exported(lib):
    syms = header_symbols()
    assert len(syms) >= 14
    assert sorted(L.EXPORTS) == syms
    for s in syms:
        assert hasattr(lib, s), s


def test_status_strings(lib):
    for code, name in L.STATUS.items():
        assert lib.tk_status_string(code).decode() == name


def _drv(lib, fn, adt=1, N=3, dims=(8, 9, 10), ranks=(2, 3, 4), opts=None, ws_bytes=1 << 30,
         ws=FAKE, A=FAKE, U=None, G=FAKE):
    U = U if U is not None else L.ptrarr([0x100000] * max(N, 1))
    return fn(A, adt, N, L.i64arr(dims) if dims is not None else None,
              L.i32arr(ranks) if ranks is not None else None,
              ctypes.byref(opts) if opts is not None else None, U, G, ws, ws_bytes, None,
              None)


@pytest.mark.parametrize("name", ["als_sthosvd", "als_thosvd"])
def test_driver_validation(lib, name):
    fn = getattr(lib, name)
    assert _drv(lib, fn, adt=7) == -2
    assert _drv(lib, fn, A=None) == -1
    assert _drv(lib, fn, G=None) == -1
    assert _drv(lib, fn, U=L.ptrarr([0x100000, 0, 0x100000])) == -1
    assert _drv(lib, fn, N=0, dims=(), ranks=()) == -1
    assert _drv(lib, fn, N=9, dims=(2,) * 9, ranks=(1,) * 9) == -1
    assert _drv(lib, fn, dims=(8, 0, 10)) == -1
    assert _drv(lib, fn, ranks=(9, 3, 4)) == -1          # R_n > I_n
    assert _drv(lib, fn, ranks=(0, 3, 4)) == -1
    assert _drv(lib, fn, ranks=(2, 3, 7)) == -1          # R_3 > R_1 R_2
    assert _drv(lib, fn, ranks=None) == -1
    assert _drv(lib, fn, ws_bytes=16) == -3
    assert _drv(lib, fn, ws=None) == -3
    o = L.tk_als_opts()
    o.struct_size = ctypes.sizeof(o)
    o.tol = -1.0
    assert _drv(lib, fn, opts=o) == -1
    o.tol = 1e-4
    o.max_iters = -3
    assert _drv(lib, fn, opts=o) == -1
    o.max_iters = 5
    o.resid_mode = 4
    assert _drv(lib, fn, opts=o) == -1
    o.resid_mode = 0
    o.compute = 1                                       # only TK_COMPUTE_AS_STORAGE
    assert _drv(lib, fn, opts=o) == -2
    o.compute = 0
    o.struct_size = 8
    assert _drv(lib, fn, opts=o) == -1
    # R_n <= 64: the r x r small linear algebra runs in one workgroup
    assert _drv(lib, fn, dims=(70, 70, 3), ranks=(65, 65, 2)) == -1
    assert _drv(lib, fn, dims=(70, 70, 3), ranks=(64, 64, 2), ws_bytes=16) == -3


def test_bad_order(lib):
    o = L.tk_als_opts()
    o.struct_size = ctypes.sizeof(o)
    o.tol = 1e-4
    o.max_iters = 5
    for bad in ([0, 0, 1], [0, 1, 3], [-1, 0, 1]):
        keep = L.i32arr(bad)
        o.order = ctypes.cast(keep, ctypes.POINTER(ctypes.c_int32))
        assert _drv(lib, lib.als_sthosvd, opts=o) == -1


def test_workspace_queries(lib):
    d, r = L.i64arr([20, 30, 40]), L.i32arr([4, 5, 6])
    a = lib.als_workspace_bytes(1, 1, 3, d, r)
    b = lib.als_workspace_bytes(0, 1, 3, d, r)
    assert a > 0 and b > 0
    assert lib.als_workspace_bytes(2, 1, 3, d, r) == 0
    assert lib.als_workspace_bytes(1, 9, 3, d, r) == 0
    assert lib.als_workspace_bytes(1, 1, 3, d, L.i32arr([21, 5, 6])) == 0
    # larger tensors need more workspace
    assert lib.als_workspace_bytes(1, 1, 3, L.i64arr([40, 60, 80]), r) > a
    assert lib.tucker_reconstruct_workspace_bytes(1, 3, r, d) > 0
    assert lib.tucker_reconstruct_workspace_bytes(2, 3, r, d) == 0
    assert lib.contract_allbut_workspace_bytes(1, 3, d, 1, 5) > 0
    assert lib.contract_allbut_workspace_bytes(1, 3, d, 3, 5) == 0
    assert lib.als_sthosvd_batched_workspace_bytes(
        2, L.i64arr([20, 30, 40, 16, 17, 18]), L.i32arr([4, 5, 6, 2, 2, 3])) > 0
    assert lib.als_sthosvd_batched_workspace_bytes(
        1, L.i64arr([20, 30, 40]), L.i32arr([40, 5, 6])) == 0


def test_workspace_queries_many_shapes(lib):
    """The host-side workspace carving over many shapes, orders, dtypes and
    ranks (also the body of the sanitizer run): every query is positive,
    t-HOSVD's never below the single-mode one, and growing a mode never
    shrinks it."""
    rng = np.random.default_rng(7)
    for _ in range(300):
        N = int(rng.integers(2, 7))
        dims = [int(x) for x in rng.integers(1, 300, size=N)]
        if rng.random() < 0.2:
            dims[int(rng.integers(N))] = int(rng.integers(1000, 5000))
        ranks = [int(rng.integers(1, min(d, 64) + 1)) for d in dims]
        for dt in (L.TK_F64, L.TK_F32, L.TK_BF16):
            st = lib.als_workspace_bytes(1, dt, N, L.i64arr(dims), L.i32arr(ranks))
            t = lib.als_workspace_bytes(0, dt, N, L.i64arr(dims), L.i32arr(ranks))
            # a Tucker core needs R_n <= prod_{k != n} R_k; other ranks are rejected
            valid = all(ranks[n] <= np.prod([ranks[k] for k in range(N) if k != n])
                        for n in range(N))
            assert (st > 0) == valid and (t > 0) == valid, (dims, ranks, dt)
            if not valid:
                continue
            grown = list(dims)
            grown[0] += 17
            assert lib.als_workspace_bytes(1, dt, N, L.i64arr(grown), L.i32arr(ranks)) >= st
            rq = lib.tucker_reconstruct_workspace_bytes(dt, N, L.i32arr(ranks), L.i64arr(dims))
            # (the reconstruction takes FP64 or FP32 cores and factors only)
            assert (rq > 0) == (dt != L.TK_BF16), (dims, ranks, dt)


def test_ttm_validation(lib):
    d = L.i64arr([4, 5, 6])
    assert lib.ttm(FAKE, 1, 3, d, 1, FAKE, 0, 3, 0, FAKE, 1, None) == -2   # M dtype
    assert lib.ttm(FAKE, 2, 3, d, 1, FAKE, 1, 3, 0, FAKE, 2, None) == -2   # bf16 out
    assert lib.ttm(FAKE, 1, 3, d, 3, FAKE, 1, 3, 0, FAKE, 1, None) == -1   # mode
    assert lib.ttm(FAKE, 1, 3, d, 1, FAKE, 1, 0, 0, FAKE, 1, None) == -1   # J
    assert lib.ttm(FAKE, 1, 3, d, 1, FAKE, 1, 3, 2, FAKE, 1, None) == -1   # trans
    assert lib.ttm(None, 1, 3, d, 1, FAKE, 1, 3, 0, FAKE, 1, None) == -1


def test_reconstruct_contract_step_validation(lib):
    d, r = L.i64arr([4, 5, 6]), L.i32arr([2, 2, 2])
    U = L.ptrarr([0x100000] * 3)
    assert lib.tucker_reconstruct(FAKE, 2, 3, r, d, U, FAKE, FAKE, 1 << 20, None) == -2
    assert lib.tucker_reconstruct(FAKE, 1, 3, r, d, U, FAKE, FAKE, 4, None) == -3
    assert lib.tucker_reconstruct(FAKE, 1, 3, r, d, L.ptrarr([0x100000, 0, 0x100000]),
                                  FAKE, FAKE, 1 << 20, None) == -1
    assert lib.contract_allbut(FAKE, FAKE, 1, 3, d, 0, 3, FAKE, FAKE, 4, None) == -3
    assert lib.contract_allbut(FAKE, FAKE, 2, 3, d, 0, 3, FAKE, FAKE, 1 << 20, None) == -2
    n2 = ctypes.c_double()
    assert lib.als_init_step(FAKE, 1, 3, d, 0, 5, 0, FAKE, FAKE, ctypes.byref(n2), FAKE,
                             1 << 30, None) == -1          # R > I_mode
    assert lib.als_init_step(FAKE, 1, 3, d, 0, 2, 0, FAKE, FAKE, ctypes.byref(n2), FAKE,
                             16, None) == -3
    assert lib.als_sweep_step(FAKE, 1, 3, d, 1, 2, FAKE, FAKE, 1.0, 3, ctypes.byref(n2), FAKE,
                              1 << 30, None) == -1         # resid mode
    assert lib.als_sweep_step(FAKE, 1, 3, d, 1, 2, FAKE, FAKE, 1.0, L.TK_RESID_AUTO,
                              ctypes.byref(n2), FAKE, 1 << 30, None) == -1   # AUTO: drivers only
    assert lib.qr_f64(FAKE, 3, 4, FAKE, None, FAKE, 1 << 20, None) == -1   # r > m
    assert lib.qr_f64(FAKE, 30, 4, FAKE, FAKE, FAKE, 1 << 20, None) == -1  # Rhat reserved
    assert lib.qr_f64(FAKE, 100, 65, FAKE, None, FAKE, 1 << 20, None) == -1  # r > 64
    assert lib.contract_allbut(FAKE, FAKE, 1, 3, L.i64arr([4, 5, 70]), 2, 65, FAKE, FAKE,
                               1 << 30, None) == -1       # J > 64
    assert lib.qr_f64(FAKE, 30, 4, FAKE, None, FAKE, 16, None) == -3


def test_batched_validation(lib):
    d3, r3 = L.i64arr([8, 9, 10]), L.i32arr([2, 3, 4])
    off = L.i64arr([0])
    u_off = L.i64arr([0, 16, 43])
    assert lib.als_sthosvd_batched(FAKE, 0, 1, d3, r3, off, None, FAKE, u_off, FAKE, off, None,
                                   None, FAKE, 1 << 30, None) == -2
    assert lib.als_sthosvd_batched(FAKE, 1, 0, d3, r3, off, None, FAKE, u_off, FAKE, off, None,
                                   None, FAKE, 1 << 30, None) == -1
    assert lib.als_sthosvd_batched(FAKE, 1, 1, d3, r3, off, None, FAKE, u_off, FAKE, off, None,
                                   None, FAKE, 8, None) == -3


def test_product_path_does_not_touch_oracle():
    """The product package never imports the oracle."""
    pkg = os.path.join(ROOT, "paper_2004_02583_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in txt.replace("oracle-free", ""), f


def test_st_order_auto_host(lib):
    """The automatic st-HOSVD order is host logic: it runs without a GPU and equals the
    oracle's exhaustive eq. 2.2 minimiser (integers, compared exactly)."""
    from oracle import tucker_oracle as o
    rng = np.random.default_rng(60)
    for N in (1, 2, 3, 4, 5, 6):
        for _ in range(6):
            dims = [int(x) for x in rng.integers(2, 200, N)]
            while True:
                ranks = [int(rng.integers(1, min(d, 64) + 1)) for d in dims]
                others_ok = all(N == 1 or ranks[n] <= int(np.prod(
                    [ranks[k] for k in range(N) if k != n])) for n in range(N))
                if others_ok:
                    break
            out = L.i32arr([0] * N)
            assert lib.st_order_auto(N, L.i64arr(dims), L.i32arr(ranks), out) == 0
            assert list(out) == o.st_order_auto(dims, ranks), (dims, ranks)
    out = L.i32arr([0] * 3)
    assert lib.st_order_auto(3, L.i64arr((8, 9, 10)), L.i32arr((9, 3, 4)), out) == -1
    assert lib.st_order_auto(3, L.i64arr((8, 9, 10)), L.i32arr((2, 3, 4)), None) == -1
    assert lib.st_order_auto(0, L.i64arr((8,)), L.i32arr((2,)), out) == -1
    # largest shape the library accepts: 8 modes, ranks 64, no overflow of the cost
    big = [230] * 8
    out8 = L.i32arr([0] * 8)
    assert lib.st_order_auto(8, L.i64arr(big), L.i32arr([64] * 7 + [63]), out8) == 0
    assert list(out8) == o.st_order_auto(big, [64] * 7 + [63])


def test_hooi_validation(lib):
    """hooi_refine rejects bad arguments before any device work."""
    dims, ranks = L.i64arr((8, 9, 10)), L.i32arr((2, 3, 4))
    U = L.ptrarr([0x100000] * 3)

    def call(adt=1, A=FAKE, N=3, d=dims, r=ranks, tol=1e-8, it=5, U=U, G=FAKE, ws=FAKE,
             wsb=1 << 30):
        return lib.hooi_refine(A, adt, N, d, r, None, tol, it, U, G, ws, wsb, None, None)
    assert call(adt=7) == -2
    assert call(A=None) == -1
    assert call(G=None) == -1
    assert call(U=L.ptrarr([0x100000, 0, 0x100000])) == -1
    assert call(tol=-1.0) == -1
    assert call(tol=float("nan")) == -1
    assert call(it=-1) == -1
    assert call(r=L.i32arr((9, 3, 4))) == -1
    assert call(wsb=16) == -3
    assert call(ws=None) == -3
    need = lib.hooi_workspace_bytes(1, 3, dims, ranks)
    assert need >= lib.als_workspace_bytes(1, 1, 3, dims, ranks)
    assert lib.hooi_workspace_bytes(1, 3, dims, L.i32arr((9, 3, 4))) == 0


def test_struct_layout_matches_header(tmp_path):
    """The ctypes structures of the binding have the header's layout: a C
    program compiled against include/tucker_als.h prints sizeof and every
    field offset."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"tk_als_opts": L.tk_als_opts, "tk_als_info": L.tk_als_info,
               "tk_hooi_info": L.tk_hooi_info}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "tucker_als.h"',
             "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{name} {fname} %zu\\n", offsetof({name}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    str(src), "-o", str(exe)], check=True)
    got = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    want = []
    for name, cls in structs.items():
        want.append(f"{name} size {ctypes.sizeof(cls)}")
        for fname, _ in cls._fields_:
            want.append(f"{name} {fname} {getattr(cls, fname).offset}")
    assert [g for g in got if g] == want


def test_enum_values_match_header():
    """Status, dtype and residual-mode values of the binding equal the header's."""
    src = open(HEADER).read()
    vals = {m.group(1): int(m.group(2)) for m in re.finditer(r"\b(TK_[A-Z0-9_]+)\s*=\s*(-?\d+)", src)}
    assert vals["TK_F64"] == L.TK_F64 and vals["TK_F32"] == L.TK_F32 and vals["TK_BF16"] == L.TK_BF16
    assert vals["TK_RESID_AUTO"] == L.TK_RESID_AUTO
    assert vals["TK_RESID_TRACE"] == L.TK_RESID_TRACE
    assert vals["TK_RESID_EXPLICIT"] == L.TK_RESID_EXPLICIT
    assert vals["TK_COMPUTE_AS_STORAGE"] == L.TK_COMPUTE_AS_STORAGE
    for code, name in L.STATUS.items():
        assert vals[name] == code


def test_noalloc_validation(lib):
    """The allocation-free entry point rejects bad arguments and shapes beyond its
    device array before any HIP call."""
    U = L.ptrarr([0x100000] * 3)
    d, r = L.i64arr([8, 9, 10]), L.i32arr([2, 3, 4])
    assert lib.als_sthosvd_noalloc_max_bytes() == 64 << 20
    assert lib.als_sthosvd_noalloc(FAKE, 7, 3, d, r, None, U, FAKE, None, None) == -2
    assert lib.als_sthosvd_noalloc(None, 1, 3, d, r, None, U, FAKE, None, None) == -1
    assert lib.als_sthosvd_noalloc(FAKE, 1, 3, d, L.i32arr([9, 3, 4]), None, U, FAKE, None,
                                   None) == -1
    big, rb = L.i64arr([400, 400, 400]), L.i32arr([40, 40, 40])
    assert lib.als_workspace_bytes(1, 1, 3, big, rb) > lib.als_sthosvd_noalloc_max_bytes()
    assert lib.als_sthosvd_noalloc(FAKE, 1, 3, big, rb, None, U, FAKE, None, None) == -3
