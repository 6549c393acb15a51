"""The allocation-free sweep hsw_apply_noalloc against hsw_apply, through the C ABI.

Two calls in a row on one context, the second with fewer right-hand sides
(the scratch keeps the first call's contents), each compared with hsw_apply
on the same input, in both precisions; then the rejections: 16 right-hand
sides, and a workspace larger than the scratch.
"""

import ctypes

import numpy as np
import pytest

from paper_1204_0111_amd import workloads as wl
from tests._cases import TOL, case, rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _noalloc(S, r, out):
    return S.lib.hsw_apply_noalloc(S.ctx, 0, ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                   r.shape[0], r.shape[1])


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_apply_noalloc_matches_apply_on_two_calls(prec):
    from paper_1204_0111_amd.hsweep import Solver
    P = case(n=(14, 12, 13), gamma=3, d=3, leaf=4)
    S = Solver(P, precision=prec)
    S.set_option("autotune", 0)  # both entry points on the fixed block shapes
    # and on the single-vector passes (hsw_apply_noalloc always takes them;
    # hsw_apply would take the matrix-core passes from 4 right-hand sides)
    S.set_option("mm_min_rhs", 16)
    S.assemble(P["c"])
    S.setup()
    n = S.N_pad()
    for nrhs, seed in ((5, 60), (3, 61), (1, 62)):
        r = torch.as_tensor(wl.random_complex((nrhs, n), seed)).to("cuda")
        ref = S.apply(0, r).cpu().numpy()
        out = torch.full((nrhs, n), float("nan"), dtype=torch.complex128, device="cuda")
        assert _noalloc(S, r, out) == 0, S.lib.hsw_last_error(S.ctx)
        got = out.cpu().numpy()
        for k in range(nrhs):
            assert rel(got[k], ref[k]) <= TOL[prec], (nrhs, k)
        assert np.array_equal(got, ref)  # the same kernels and shapes: bit for bit
    S.close()


def test_apply_noalloc_rejects_sizes_past_its_limits():
    from paper_1204_0111_amd.hsweep import Solver
    P = case(n=(14, 12, 13), gamma=3, d=3, leaf=4)
    S = Solver(P, precision="c64")
    S.assemble(P["c"])
    S.setup()
    n = S.N_pad()
    r = torch.zeros((16, n), dtype=torch.complex128, device="cuda")
    out = torch.zeros_like(r)
    assert _noalloc(S, r, out) == 1  # HSW_E_INVAL: at most 15 right-hand sides per call
    assert b"at most 15" in S.lib.hsw_last_error(S.ctx)
    S.close()
    # the 100^3 layered workload needs about 19 MB of complex64 workspace per
    # right-hand side: 15 of them do not fit the 128 MiB scratch
    Q = wl.make_problem("layered100")
    S = Solver(Q, precision="c64")
    S.assemble(Q["c"])
    S.setup()
    n = S.N_pad()
    r = torch.zeros((15, n), dtype=torch.complex128, device="cuda")
    out = torch.zeros_like(r)
    assert _noalloc(S, r, out) == 1
    assert b"scratch" in S.lib.hsw_last_error(S.ctx)
    # and one right-hand side does fit, and matches hsw_apply
    r1 = torch.as_tensor(wl.random_complex((1, n), 63)).to("cuda")
    out1 = torch.empty_like(r1)
    assert _noalloc(S, r1, out1) == 0, S.lib.hsw_last_error(S.ctx)
    ref = S.apply(0, r1).cpu().numpy()
    assert rel(out1.cpu().numpy()[0], ref[0]) <= TOL["c64"]
    S.close()
