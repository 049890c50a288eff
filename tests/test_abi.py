"""C-ABI checks that need no GPU: the library loads, exports every entry point
that include/teno.h declares, the ctypes mirrors match the C struct layout,
and host-side validation rejects bad arguments before anything is enqueued."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "teno.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:[A-Za-z_][\w\s\*]*?)\b(teno_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def B():
    from paper_2003_09145_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libteno.so not built")
    binding.lib()
    return binding


def test_header_declares_the_entry_points():
    names = declared_functions()
    for f in ("teno_rhs", "teno_step", "teno_workspace_bytes", "teno_ctrl_init"):
        assert f in names


def test_library_exports_every_declared_symbol(B):
    L = ctypes.CDLL(B.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name
    assert sorted(B.SYMBOLS) == sorted(n for n in declared_functions() if n in B.SYMBOLS)
    assert set(declared_functions()) <= set(B.SYMBOLS)


def test_struct_layout_matches_header(tmp_path, B):
    prog = tmp_path / "layout.c"
    prog.write_text(r"""
#include <stdio.h>
#include <stddef.h>
#include "teno.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(teno_grid), offsetof(teno_grid, dx),
         offsetof(teno_grid, bc), offsetof(teno_grid, gamma), offsetof(teno_grid, H),
         offsetof(teno_grid, Bl), offsetof(teno_grid, eps), offsetof(teno_grid, flags),
         offsetof(teno_grid, a1), offsetof(teno_grid, xi));
  printf("%zu %zu %zu %zu %zu %zu %d %d\n", sizeof(teno_side), sizeof(teno_boundary),
         offsetof(teno_boundary, gravity), offsetof(teno_side, state), offsetof(teno_grid, boundary_dev),
         offsetof(teno_grid, theta), TENO_THETA_PRINTED, TENO_THETA_CUT);
  printf("%zu %zu %zu %zu %zu\n", sizeof(teno_ctrl), offsetof(teno_ctrl, alpha),
         offsetof(teno_ctrl, status), offsetof(teno_ctrl, nsteps), offsetof(teno_ctrl, active));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    G, C = B.TenoGrid, B.TenoCtrl
    assert [int(x) for x in out[0].split()] == [
        ctypes.sizeof(G), G.dx.offset, G.bc.offset, G.gamma.offset, G.H.offset, G.Bl.offset,
        G.eps.offset, G.flags.offset, G.a1.offset, G.xi.offset]
    Sd, Bd = B.TenoSide, B.TenoBoundary
    assert [int(x) for x in out[1].split()] == [
        ctypes.sizeof(Sd), ctypes.sizeof(Bd), Bd.gravity.offset, Sd.state.offset,
        G.boundary_dev.offset, G.theta.offset, B.THETA["printed"], B.THETA["cut"]]
    assert [int(x) for x in out[2].split()] == [
        ctypes.sizeof(C), C.alpha.offset, C.status.offset, C.nsteps.offset, C.active.offset]


def _grid(B, **kw):
    prob = dict(ndim=2, n=[16, 12], dx=[0.1, 0.1], bc="periodic")
    prob.update(kw)
    return B.grid(prob)


def test_workspace_bytes(B):
    g = _grid(B)
    nb = B.lib().teno_workspace_bytes(ctypes.byref(g))
    assert nb >= 3 * 4 * 16 * 12 * 8
    bad = _grid(B, n=[2, 12])
    assert B.lib().teno_workspace_bytes(ctypes.byref(bad)) == 0


@pytest.mark.parametrize("kw", [
    dict(ndim=0), dict(ndim=4, n=[8, 8, 8, 8]), dict(n=[2, 12]), dict(dx=[0.0, 0.1]),
    dict(dx=[0.1, -1.0]), dict(bc=[7, 0]), dict(gamma=1.0), dict(scheme=5),
    dict(Bl=5, Bu=4), dict(Bu=21), dict(H=0.0), dict(eps=0.0),
    dict(scheme="teno5a", a1=3.0, a2=3.5), dict(scheme="teno5a", a1=21.0),
    dict(scheme="teno5a", cr=0.0), dict(scheme="teno5a", cr=1.2), dict(scheme="teno5a", xi=-1.0),
    dict(scheme="teno5a", a2=-1.0), dict(theta=2), dict(theta=-1)])
def test_validation_rejects_bad_grids(B, kw):
    try:
        g = _grid(B, **kw)
    except (IndexError, KeyError):
        return
    L = B.lib()
    dummy = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    assert L.teno_rhs(ctypes.byref(g), dummy, dummy, None, None, None, dummy, 1 << 40, None) == B.ERR_ARG
    assert L.teno_step(ctypes.byref(g), dummy, dummy, dummy, 1 << 40, None) == B.ERR_ARG


def test_validation_rejects_null_buffers_and_small_workspace(B):
    g = _grid(B)
    L = B.lib()
    d = ctypes.c_void_p(0x1000)
    nb = L.teno_workspace_bytes(ctypes.byref(g))
    assert L.teno_rhs(ctypes.byref(g), None, d, None, None, None, d, nb, None) == B.ERR_ARG
    assert L.teno_rhs(ctypes.byref(g), d, None, None, None, None, d, nb, None) == B.ERR_ARG
    assert L.teno_rhs(ctypes.byref(g), d, d, None, None, None, None, nb, None) == B.ERR_ARG
    assert L.teno_rhs(ctypes.byref(g), d, d, None, None, None, d, nb - 1, None) == B.ERR_ARG
    assert L.teno_step(ctypes.byref(g), d, None, d, nb, None) == B.ERR_ARG
    assert L.teno_rhs_debug(ctypes.byref(g), d, d, None, None, None, None, d, nb, None) == B.ERR_ARG
    assert L.teno_ctrl_init(None, 0.0, 1.0, 0.5, None) == B.ERR_ARG
    assert L.teno_ctrl_init(d, 0.0, 1.0, 0.0, None) == B.ERR_ARG
