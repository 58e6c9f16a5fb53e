"""GPU: the continuous-batching runtime (cmb_server_*) against one-request
solves through cmb_solve.  A request's spectrum must not depend on its batch
mates, the batch size or the stream it ran on: every comparison is bitwise."""
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


def _mixed_requests(n, seed=7):
    """Requests of one small hierarchy (photon/massless cut 8, polarisation)
    with mixed k grids, output-time counts and ell_max."""
    base = W.small_case(n_k=10, n_tau=150, ell_max=60)
    cos = W.perturbed_cosmologies(n, seed=seed)
    shapes = [(10, 150, 60), (16, 120, 120), (24, 200, 200)]
    out = []
    for i in range(n):
        c = cos[i]
        c["N_nu_massless"] = 3.0
        nk, nt, lm = shapes[i % 3]
        out.append(dict(cosmo=c, prec=dict(base.prec), k=W.log_grid(1e-4, 0.05 * lm / 60, nk), n_tau=nt,
                        ell_max=lm))
    return out


def _alone(ctx, r):
    import torch
    import paper_2602_15104_amd as L
    tab = L.Tables(r["cosmo"], r["prec"], r["k"], r["n_tau"])
    out = L.solve_batch(ctx, [tab], r["ell_max"], keep_S=False, keep_Delta=False)
    torch.cuda.synchronize()
    return out["Cl"][0].cpu().numpy(), out["status"][0].cpu().numpy()


@pytest.fixture(scope="module")
def ctx():
    _need_gpu()
    import paper_2602_15104_amd as L
    c = L.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("max_batch,n_streams", [(4, 2), (1, 1), (64, 4)])
def test_serving_matches_alone(ctx, max_batch, n_streams):
    import paper_2602_15104_amd as L
    reqs = _mixed_requests(9)
    _say("serving", len(reqs), "requests, max_batch", max_batch, "streams", n_streams)
    srv = L.Server(0, n_workers=3, n_streams=n_streams, max_batch=max_batch, hbm_budget_bytes=1 << 30)
    try:
        tickets = [srv.submit(r["cosmo"], r["prec"], r["k"], r["n_tau"], r["ell_max"]) for r in reqs]
        got = [srv.wait(t, timeout_s=120.0) for t in tickets]
    finally:
        srv.close()
    for r, (Cl, st, tm) in zip(reqs, got):
        ref, st_ref = _alone(ctx, r)
        assert np.all(st == 0) and np.array_equal(st, st_ref)
        assert np.array_equal(Cl, ref), np.max(np.abs(Cl - ref))
        assert 0.0 <= tm["submit"] <= tm["tables_ready"] <= tm["launched"] <= tm["done"]
        assert 1 <= tm["batch_size"] <= max_batch
    # the mix really happened: requests shared a batch, and batches on
    # different streams were on the device at the same time (one batch per
    # launch time; a batch launched before an earlier one finished overlaps it)
    times = [tm for _, _, tm in got]
    sizes = [tm["batch_size"] for tm in times]
    batches = sorted({(tm["launched"], tm["done"]) for tm in times})
    overlaps = sum(1 for i in range(1, len(batches)) if batches[i][0] < max(d for _, d in batches[:i]))
    _say("batch sizes", sizes, "batches", len(batches), "overlapping launches", overlaps)
    if max_batch == 1:
        assert max(sizes) == 1 and overlaps == 0
    else:
        assert max(sizes) > 1
        assert overlaps >= 1


def test_serving_rejects_other_hierarchy():
    _need_gpu()
    import paper_2602_15104_amd as L
    reqs = _mixed_requests(2)
    srv = L.Server(0, hbm_budget_bytes=1 << 28)
    try:
        t = srv.submit(reqs[0]["cosmo"], reqs[0]["prec"], reqs[0]["k"], reqs[0]["n_tau"], reqs[0]["ell_max"])
        p = dict(reqs[1]["prec"])
        p["ell_gamma"] = p["ell_gamma"] + 2
        with pytest.raises(L.CmbError) as e:
            srv.submit(reqs[1]["cosmo"], p, reqs[1]["k"], reqs[1]["n_tau"], reqs[1]["ell_max"])
        assert e.value.name == "CMB_E_INVALID"
        srv.wait(t, timeout_s=120.0)
    finally:
        srv.close()


def test_serving_reports_table_errors():
    """A request whose host tables cannot be built completes with the
    builder's error; the others are unaffected."""
    _need_gpu()
    import paper_2602_15104_amd as L
    reqs = _mixed_requests(3)
    bad = dict(reqs[1]["cosmo"])
    bad["h"] = -0.7
    srv = L.Server(0, hbm_budget_bytes=1 << 28)
    try:
        t0 = srv.submit(reqs[0]["cosmo"], reqs[0]["prec"], reqs[0]["k"], reqs[0]["n_tau"], reqs[0]["ell_max"])
        t1 = srv.submit(bad, reqs[1]["prec"], reqs[1]["k"], reqs[1]["n_tau"], reqs[1]["ell_max"])
        t2 = srv.submit(reqs[2]["cosmo"], reqs[2]["prec"], reqs[2]["k"], reqs[2]["n_tau"], reqs[2]["ell_max"])
        with pytest.raises(L.CmbError) as e:
            srv.wait(t1, timeout_s=120.0)
        assert e.value.name == "CMB_E_INVALID"
        for t in (t0, t2):
            Cl, st, _ = srv.wait(t, timeout_s=120.0)
            assert np.all(st == 0) and np.all(np.isfinite(Cl))
    finally:
        srv.close()


def test_serving_config3_requests(ctx):
    """Six requests of the Poisson serving workload (C1 physics, ell_max in
    {500, 1000, 2500} with 100/250/400 modes, 2000 output times) in one
    server: each equals its solo solve bitwise."""
    import paper_2602_15104_amd as L
    reqs = W.serving_requests(6, seed=20260215)
    prec = W.config1().prec
    srv = L.Server(0, n_workers=4, n_streams=2, max_batch=64, hbm_budget_bytes=2 << 30)
    try:
        tickets = [srv.submit(r["cosmo"], prec, r["k"], 2000, r["ell_max"]) for r in reqs]
        got = [srv.wait(t, timeout_s=120.0) for t in tickets]
    finally:
        srv.close()
    for r, (Cl, st, tm) in zip(reqs, got):
        ref, _ = _alone(ctx, dict(cosmo=r["cosmo"], prec=prec, k=r["k"], n_tau=2000, ell_max=r["ell_max"]))
        _say("request l_max", r["ell_max"], "n_k", len(r["k"]), "latency ms", 1e3 * (tm["done"] - tm["submit"]),
             "batch", tm["batch_size"])
        assert np.all(st == 0)
        assert np.array_equal(Cl, ref)
