"""fl_apply_D_noalloc (the entry point for callers that cannot allocate)
through the C ABI against fl_apply_D on the same device spinors: the same
kernels run, so the results agree bit for bit; two calls in a row, the
second with fewer right-hand sides (the fixed scratch array keeps the first
call's contents), and requests beyond the array are rejected on the host."""
import ctypes

import numpy as np
import pytest

import oracle as O
import synth_inputs as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import paper_1108_2473_amd as fl
    fl.lib()
    return fl


@pytest.mark.parametrize("dagger", [False, True])
def test_noalloc_apply_D_matches_apply_D(F, dagger):
    import torch
    dims, bc, kappa = (8, 8, 8, 16), -1, 0.13
    U = S.random_links(dims, 0.5, 4321)
    lat = F.Lattice(dims, bc)
    lat.set_gauge(U)
    lat.set_kappa(kappa)
    try:
        V = S.volume(dims)
        # 64 MiB of scratch hold nrhs * V * 384 bytes: 21 spinors of 8^3 x 16
        assert 21 * V * 384 <= 64 << 20 < 22 * V * 384
        for nrhs, seed in ((16, 11), (3, 12)):
            psi = torch.from_numpy(S.random_spinors(dims, nrhs, seed)).cuda()
            out = torch.full_like(psi, complex(np.nan, np.nan))
            lat.apply_D_noalloc(psi, out, dagger=dagger)
            torch.cuda.synchronize()
            ref = lat.apply_D(psi, dagger=dagger)
            torch.cuda.synchronize()
            assert torch.equal(out, ref)
            want = O.apply_D(U, psi.cpu().numpy(), dims, bc, kappa, dagger=dagger)
            assert np.abs(out.cpu().numpy() - want).max() <= 1e-13 * np.abs(want).max()
        # beyond the scratch array: FL_ERR_ARG before any launch
        big = torch.zeros((22, V, 4, 3), dtype=torch.complex128, device="cuda")
        st = F.lib().fl_apply_D_noalloc(lat._h, ctypes.c_void_p(big.data_ptr()), ctypes.c_void_p(big.data_ptr()),
                                        22, 0)
        assert st == -1 and b"MiB" in F.lib().fl_last_error(lat._h)
    finally:
        lat.close()
