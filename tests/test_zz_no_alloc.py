"""GPU: cmb_solve_noalloc, the whole path with every intermediate in the
library's fixed device array, against cmb_solve (the same kernels with
context buffers).  Results must be the same bits; the call must allocate no
device memory; a batch beyond the fixed array is refused with its outputs
untouched."""
import numpy as np
import pytest

import cmb_workloads as W

pytestmark = pytest.mark.gpu


def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _say(*a):
    print(*a, flush=True)


def _tables(wl, n, seed):
    import paper_2602_15104_amd as L
    cos = W.perturbed_cosmologies(n, seed=seed)
    for c in cos:
        c["N_nu_massless"] = 3.0
    return [L.Tables(c, wl.prec, wl.k, wl.n_tau) for c in cos]


def _both(ctx, tabs, ell_max):
    import torch
    import paper_2602_15104_amd as L
    n, n_k = len(tabs), len(tabs[0].export()["k"])
    ref = L.solve_batch(ctx, tabs, ell_max, keep_S=False, keep_Delta=False)
    Cl = torch.full((n, 3, ell_max + 1), -1.0, dtype=torch.float64, device="cuda:0")
    st = torch.full((n, n_k), -1, dtype=torch.int32, device="cuda:0")
    ns = torch.full((n, n_k), -1, dtype=torch.int32, device="cuda:0")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info(0)[0]
    L.solve_noalloc(tabs, ell_max, Cl, st, ns)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info(0)[0]
    return ref, (Cl, st, ns), free0 - free1


def test_noalloc_matches_solve_twice_then_smaller():
    _need_gpu()
    import torch
    import paper_2602_15104_amd as L
    assert L.noalloc_scratch_bytes() == 160 << 20
    ctx = L.Context(0)
    try:
        # first call: two config-1 cosmologies (400 modes, 2000 output times,
        # l <= 2500; 72 MiB of intermediates); second: a smaller batch
        big = W.config1()
        small = W.small_case(n_k=9, n_tau=90, ell_max=50)
        cases = [(big, _tables(big, 2, 11)), (small, _tables(small, 3, 12)), (small, _tables(small, 1, 13))]
        for i, (wl, tabs) in enumerate(cases):
            _say("noalloc call", i, wl.name, "batch", len(tabs))
            ref, (Cl, st, ns), used = _both(ctx, tabs, wl.ell_max)
            assert torch.equal(ref["Cl"], Cl)
            assert torch.equal(ref["status"], st) and torch.all(st == 0)
            assert torch.equal(ref["nsteps"], ns)
            if i > 0:  # the fixed array exists after the first call on the device
                assert used == 0, used
        # beyond the fixed array: refused, outputs untouched
        tabs = _tables(big, 5, 14)
        Cl = torch.full((5, 3, big.ell_max + 1), -1.0, dtype=torch.float64, device="cuda:0")
        st = torch.full((5, len(big.k)), -1, dtype=torch.int32, device="cuda:0")
        with pytest.raises(L.CmbError) as e:
            L.solve_noalloc(tabs, big.ell_max, Cl, st)
        assert e.value.name == "CMB_E_NOMEM"
        torch.cuda.synchronize()
        assert torch.all(Cl == -1.0) and torch.all(st == -1)
        # step counts into the fixed array when the caller passes none
        wl, tabs = cases[1]
        Cl = torch.empty((3, 3, wl.ell_max + 1), dtype=torch.float64, device="cuda:0")
        st = torch.empty((3, len(wl.k)), dtype=torch.int32, device="cuda:0")
        L.solve_noalloc(tabs, wl.ell_max, Cl, st)
        ref = L.solve_batch(ctx, tabs, wl.ell_max, keep_S=False, keep_Delta=False)
        torch.cuda.synchronize()
        assert torch.equal(ref["Cl"], Cl)
    finally:
        ctx.close()
