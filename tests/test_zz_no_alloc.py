"""The classification entry point that allocates nothing (ibm_classify_noalloc) equals the
handle's ibm_classify: the same cell types, bit for bit, and the same counts, on two calls
in a row through the C ABI, the second on a smaller grid (the static scratch keeps the first
call's contents, which must not leak into the second)."""
import ctypes as C

import numpy as np
import pytest

from paper_2505_17287_amd import ibm
from paper_2505_17287_amd import inputs as I


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _noalloc(torch, wl, type_out):
    nx, ny, nz = wl.shape
    dev = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda() for a in (wl.xf, wl.yf, wl.zf)]
    verts = torch.from_numpy(np.ascontiguousarray(wl.verts, dtype=np.float64)).cuda()
    tris = torch.from_numpy(np.ascontiguousarray(wl.tris, dtype=np.int32)).cuda()
    counts = np.zeros(3, np.int64)
    stream = torch.cuda.current_stream()
    code = ibm.lib().ibm_classify_noalloc(nx, ny, nz, *[C.c_void_p(a.data_ptr()) for a in dev],
                                          C.c_void_p(verts.data_ptr()), len(wl.verts), C.c_void_p(tris.data_ptr()),
                                          len(wl.tris), C.c_void_p(type_out.data_ptr()), C.c_void_p(counts.ctypes.data),
                                          C.c_void_p(stream.cuda_stream))
    return code, counts


@pytest.mark.gpu
def test_classify_noalloc_equals_ibm_classify_twice():
    torch = _torch()
    cases = (I.multibody(128, n_bodies=4, level=4), I.wing(96, 48, 40))  # the second is smaller
    for wl in cases:
        print("noalloc case", wl.name, flush=True)
        g = ibm.Grid(wl.xf, wl.yf, wl.zf)
        try:
            ref_counts = g.setup(wl.verts, wl.tris)
            ref = g.cell_types()
        finally:
            g.close()
        nx, ny, nz = wl.shape
        out = torch.full((nz, ny, nx), 0xAB, dtype=torch.uint8, device="cuda")
        code, counts = _noalloc(torch, wl, out)
        assert code == ibm.IBM_OK, ibm.lib().ibm_last_error(None)
        assert torch.equal(out, ref)
        assert tuple(counts) == tuple(int(c) for c in ref_counts)
