"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol the header declares, reports its version, implements the keyed
generator exactly as the oracle's written specification, and rejects invalid
arguments before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tsk.h")


def _lib():
    from paper_2104_01101_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libtsk.so not built")
    return L


def test_header_symbols_exported():
    L = _lib()
    lib = L.lib()
    names = re.findall(r"\b(tsk_[a-z0-9_]+)\s*\(", open(HEADER).read())
    assert len(set(names)) >= 18
    for n in set(names):
        assert hasattr(lib, n), n


def test_abi_version():
    """Version 5: the options struct gained first_sweep and tol (resume and
    convergence test of the sweep loop) and the FINAL_FIT flag."""
    L = _lib()
    assert L.lib().tsk_abi_version() == 5


def test_options_layout_matches_header(tmp_path):
    """The ctypes mirror of tsk_options and tsk_tensor has the C compiler's
    offsets and sizes (a C program built against include/tsk.h prints them)."""
    import shutil
    import subprocess
    L = _lib()
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    opt_fields = [f for f, _ in L._Options._fields_]
    ten_fields = [f for f, _ in L._Tensor._fields_]
    src = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"',
           'int main(void) {',
           '  printf("%zu %zu\\n", sizeof(tsk_options), sizeof(tsk_tensor));']
    src += [f'  printf("%zu\\n", offsetof(tsk_options, {f}));' for f in opt_fields]
    src += [f'  printf("%zu\\n", offsetof(tsk_tensor, {f}));' for f in ten_fields]
    src += ['  return 0;', '}']
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", str(c), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    sizes, offs = [int(v) for v in out[:2]], [int(v) for v in out[2:]]
    assert sizes == [ctypes.sizeof(L._Options), ctypes.sizeof(L._Tensor)]
    want = [getattr(L._Options, f).offset for f in opt_fields] + \
        [getattr(L._Tensor, f).offset for f in ten_fields]
    assert offs == want


def test_generator_matches_oracle_spec():
    L = _lib()
    from oracle import rng
    lib = L.lib()
    for seed, purpose, a, b, c in [(0, -1, 0, 0, 0), (7, 1, 2, 0, 0), (123, 4, 3, 1, 2)]:
        k_lib = lib.tsk_stream_key(seed, purpose, a, b, c)
        k_or = int(rng.stream_key(seed, None if purpose < 0 else purpose, a, b, c)[0])
        assert k_lib == k_or
        for i in (0, 1, 17, 123456789):
            assert lib.tsk_draw(k_lib, i) == int(rng.draw(k_or, [i])[0])


def _tensor(L, dims, layout=0, dtype=1, nnz=0):
    t = L._Tensor()
    t.order = len(dims)
    for k, d in enumerate(dims):
        t.dims[k] = d
    t.dtype, t.layout, t.nnz = dtype, layout, nnz
    t.values = 1 if nnz or layout == 0 else 0
    return t


def _opts(L, m, sketch=0, solve=0, rsvd_k=0):
    o = L._Options()
    o.m, o.sketch, o.sweeps, o.prec = m, sketch, 1, 0
    o.solve, o.rsvd_k = solve, rsvd_k
    return o


@pytest.mark.parametrize("first_sweep,tol,flags,expect", [
    (0, 0.0, 0, 0),
    (3, 0.0, 0, 0),      # resume at sweep 3
    (-1, 0.0, 0, -1),    # negative first sweep
    (0, -1e-3, 1, -1),   # negative tolerance
    (0, 1e-3, 0, -1),    # tolerance without the per-sweep residual
    (0, 1e-3, 3, -1),    # tolerance with the final residual only
    (0, 1e-3, 1, 0),
])
def test_resume_and_tolerance_validation(first_sweep, tol, flags, expect):
    L = _lib()
    t = _tensor(L, (10, 10, 10))
    o = _opts(L, 50)
    o.first_sweep, o.tol, o.flags = first_sweep, tol, flags
    nb = ctypes.c_size_t(0)
    st = L.lib().tsk_workspace_size(ctypes.byref(t), L.i32_array((3, 3, 3)), ctypes.byref(o),
                                    ctypes.byref(nb))
    assert st == expect


@pytest.mark.parametrize("dims,ranks,m,sketch,layout,expect", [
    ((10, 10, 10), (3, 3, 3), 5, 0, 0, -1),        # m < prod of other ranks
    ((10, 10, 10), (11, 3, 3), 50, 0, 0, -1),      # rank above dimension
    ((10,), (3,), 50, 0, 0, -1),                   # order 1
    ((2**31 - 1,) * 3, (3, 3, 3), 50, 1, 1, -2),   # leverage on COO: fibre keys beyond 64 bits
    ((5, 5, 5), (2, 2, 2), 30, 2, 0, -1),          # deterministic selection: m > 25 rows
    ((5, 5, 5), (2, 2, 2), 30, 3, 0, -1),          # unknown sketch
    ((10, 10, 10), (3, 3, 20), 50, 0, 0, -1),      # R_n above the product of the others... and s
])
def test_validation_errors(dims, ranks, m, sketch, layout, expect):
    L = _lib()
    t = _tensor(L, dims, layout=layout, nnz=5 if layout else 0)
    if layout:
        for k in range(len(dims)):
            t.idx[k] = 8
    o = _opts(L, m, sketch)
    nb = ctypes.c_size_t(0)
    st = L.lib().tsk_workspace_size(ctypes.byref(t), L.i32_array(ranks), ctypes.byref(o),
                                    ctypes.byref(nb))
    assert st == expect
    assert len(L.lib().tsk_last_error()) > 0


def test_workspace_query_sizes_grow_with_problem():
    L = _lib()
    sizes = []
    for s in (20, 40, 80):
        t = _tensor(L, (s, s, s))
        o = _opts(L, 200)
        nb = ctypes.c_size_t(0)
        assert L.lib().tsk_workspace_size(ctypes.byref(t), L.i32_array((5, 5, 5)),
                                          ctypes.byref(o), ctypes.byref(nb)) == 0
        sizes.append(nb.value)
    assert sizes[0] < sizes[1] < sizes[2]


@pytest.mark.parametrize("solve,rsvd_k,expect", [
    (2, 0, -1),      # unknown solver
    (1, -1, -1),     # negative width
    (1, 2, -1),      # k < R
    (1, 10, -1),     # k > r = 9
    (1, 0, 0),       # default width min(R + 10, r)
    (1, 9, 0),
])
def test_rsvd_option_validation(solve, rsvd_k, expect):
    L = _lib()
    t = _tensor(L, (10, 10, 10))
    o = _opts(L, 50, 0, solve, rsvd_k)
    nb = ctypes.c_size_t(0)
    st = L.lib().tsk_workspace_size(ctypes.byref(t), L.i32_array((3, 3, 3)), ctypes.byref(o),
                                    ctypes.byref(nb))
    assert st == expect


def test_fibre_index_query_sizes():
    """Host-side size query of the fibre index (no device work): keys and values
    of every entry; the leverage job on a COO tensor holds N of them."""
    L = _lib()
    t = _tensor(L, (100, 90, 80), dtype=0, layout=1, nnz=1000)
    for k in range(3):
        t.idx[k] = 8
    ib, wb = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert L.lib().tsk_fiber_index(ctypes.byref(t), 1, None, ctypes.byref(ib), None,
                                   ctypes.byref(wb), None) == 0
    assert 1000 * (8 + 4) <= ib.value <= 1000 * (8 + 4) + 1024
    assert wb.value >= 1000 * 8
    dense = _tensor(L, (10, 10, 10))
    assert L.lib().tsk_fiber_index(ctypes.byref(dense), 0, None, ctypes.byref(ib), None,
                                   ctypes.byref(wb), None) == -1
    sizes = []
    for sketch in (0, 1):
        o = _opts(L, 200, sketch)
        nb = ctypes.c_size_t(0)
        assert L.lib().tsk_workspace_size(ctypes.byref(t), L.i32_array((5, 5, 5)),
                                          ctypes.byref(o), ctypes.byref(nb)) == 0
        sizes.append(nb.value)
    assert sizes[1] > 3 * 1000 * 12


@pytest.mark.gpu
def test_selection_workspace_query():
    """Deterministic selection sizes its candidate set on the host: m ln m
    rank tuples for three modes (here m = 1600 of 2000 x 2000 rows).  The radix
    sort's scratch size depends on the device, so the query needs the GPU."""
    L = _lib()
    t = _tensor(L, (2000, 2000, 2000), layout=1, dtype=0, nnz=1000)
    for k in range(3):
        t.idx[k] = 8
    sizes = {}
    for sketch in (1, 2):
        o = _opts(L, 1600, sketch)
        nb = ctypes.c_size_t(0)
        assert L.lib().tsk_workspace_size(ctypes.byref(t), L.i32_array((10, 10, 10)),
                                          ctypes.byref(o), ctypes.byref(nb)) == 0
        sizes[sketch] = nb.value
    ncand = sum(min(2000, 1600 // (r + 1)) for r in range(1600))   # 12.6k per mode
    assert sizes[2] - sizes[1] >= 3 * ncand * 2 * 4
