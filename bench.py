"""Benchmark: C_ell spectra/s at ell_max = 2500 in FP64, batched vs plain, with
p50/p99 solve latency, on one MI355X.

A step is one pass of the whole hot path (perturbations + sources, Bessel
recurrence + line-of-sight projection, k quadrature) over one batch of
synthetic cosmologies of the 400-mode / 2000-output-time / l <= 2500
workload (TT/TE/EE, photon T+P and massless-neutrino hierarchies cut at
l = 24).  Tables are built and uploaded before the timed region (inputs
resident in HBM).  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--batch B] [--plain-reps R]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "C_ell spectra/s at ell_max=2500 FP64, batched vs plain; p50/p99 solve latency"
FP64_PEAK_TFLOPS = 78.6  # MI355X vector FP64: 256 CU x 2.4 GHz x 128 flop/cycle


def k1_flops_per_step(N: int, n_chains: int = 3) -> float:
    """Arithmetic the perturbation kernel executes in one ESDIRK step (five
    implicit stages) of its continuant stage solve, N state rows (exp, sqrt,
    reciprocal = 1 flop):
      stage right-hand sides  sum_s 2 s N  (s = 1..5)   = 30 N
      per stage and row: continuant sweep up 6, pivot reciprocals and
      downward coefficients 5, downward sweep 2, K = (Y - R)/g 2  = 75 N
      error estimate and norm                            = 19 N
      per stage: top rows of each chain ~184, coupling solve ~150,
      background ~60                                     = 5 (184 n_chains + 210)
      step control                                       = 10"""
    return 124.0 * N + 5.0 * (184.0 * n_chains + 210.0) + 10.0


K1_FLOPS_PER_OUTPUT = 250.0  # Hermite interpolation of 12 rows + source formulas


def k1_flops_per_step_scope(N: int) -> float:
    """The algorithmic work per ESDIRK step that the hot path's scope sets for
    the structured stage solve of a banded hierarchy (bandwidth b = 3, s = 6
    stages): per implicit stage the right-hand side A y (12 N), assembling
    I - h gamma A (7 N), the banded LU (18 N), three triangular solves (36 N),
    the rank-2 Woodbury correction (6 N) and the stage combination (12 N),
    about 90 N; six stages plus the error estimate, 560 N per step.  The
    roofline fraction of the perturbation kernel is quoted on this count."""
    return 560.0 * N
K2_FLOPS_PER_TRIPLE = 13.0   # recurrence (3) + T projection (8) + E projection (2)
K2_FLOPS_PER_SEED_STEP = 3.0


def ell_act(x: np.ndarray, ell_max: int) -> np.ndarray:
    """Highest multipole the projection kernel evaluates for each x (its skip
    rule: |j_l(x)| < 1e-15 above x + 11 x^(1/3) + 12)."""
    lc = np.ceil(x + 11.0 * np.cbrt(x) + 12.0)
    la = np.minimum(lc, ell_max)
    la = np.where(x >= ell_max + 33, ell_max, la)
    return np.where(x == 0, 1, la)


def k2_flops(k: np.ndarray, chi: np.ndarray, ell_max: int) -> float:
    x = np.outer(k, chi)
    la = ell_act(x, ell_max)
    triples = np.sum(np.maximum(la - 1, 0))
    seed = np.where(x >= ell_max + 33, ell_max + 1, np.ceil(x + 16.0 * np.cbrt(x) + 24.0))
    seed = np.where(x == 0, 0, seed)
    return float(triples * K2_FLOPS_PER_TRIPLE + np.sum(seed) * K2_FLOPS_PER_SEED_STEP)


def k1_traffic(batch: int):
    """HBM bytes per batched K1 launch from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter reads
    for a plain copy of known size), or None when that summary was taken on
    other kernel sources or another batch size."""
    path = os.path.join(ROOT, "profiles", "perturb2_config1_b32_hbm.md")
    if batch != 32 or not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ": " in line and not line.startswith(("|", " ", "#", "-")):
            k, v = line.strip().split(": ", 1)
            kv[k] = v
    try:
        h = hashlib.sha256(b"".join(open(os.path.join(ROOT, f), "rb").read() for f in kv["source_files"].split()))
        if h.hexdigest() != kv["source_sha256"]:
            return None
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, OSError, ValueError):
        return None


def k_fp64_measured(batch: int):
    """FP64 operations per launch of each kernel from the committed rocprofv3
    counter summary (VALU FP64 instruction counters times the active lanes
    per instruction), or None when that summary was taken on other kernel
    sources or another batch size."""
    path = os.path.join(ROOT, "profiles", "fp64_config1_b32_counters.md")
    if batch != 32 or not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ": " in line and not line.startswith(("|", " ", "#", "-")):
            k, v = line.strip().split(": ", 1)
            kv[k] = v
    try:
        h = hashlib.sha256(b"".join(open(os.path.join(ROOT, f), "rb").read() for f in kv["source_files"].split()))
        if h.hexdigest() != kv["source_sha256"]:
            return None
        out = {}
        for k in ("perturb", "los"):
            if f"{k}_fp64_flops_per_launch" in kv:
                out[k] = {"flops_per_launch": float(kv[f"{k}_fp64_flops_per_launch"]), "what": kv.get("what", "")}
        return out or None
    except (KeyError, OSError, ValueError):
        return None


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def serve(reqs, prec, n_tau, max_batch, n_streams, n_workers=8):
    """Replay the requests' arrival times against a serving runtime; returns
    per-request latency (arrival to spectra on the host) and its parts."""
    import paper_2602_15104_amd as L
    srv = L.Server(0, n_workers=n_workers, n_streams=n_streams, max_batch=max_batch, hbm_budget_bytes=16 << 30)
    try:
        t0 = time.perf_counter()
        tickets = []
        for r in reqs:
            dt = r["arrival_s"] - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            tickets.append(srv.submit(r["cosmo"], prec, r["k"], n_tau, r["ell_max"]))
        res = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
    tm = [x[2] for x in res]
    lat = np.array([t["done"] - t["submit"] for t in tm]) * 1e3
    span = max(t["done"] for t in tm) - min(t["submit"] for t in tm)
    bad = sum(int(np.any(x[1] != 0)) for x in res)
    return {"requests": len(reqs), "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "mean_ms": float(lat.mean()),
            "max_ms": float(lat.max()), "throughput_per_s": len(reqs) / span,
            "mean_tables_ms": 1e3 * float(np.mean([t["tables_ready"] - t["submit"] for t in tm])),
            "mean_queue_ms": 1e3 * float(np.mean([t["launched"] - t["tables_ready"] for t in tm])),
            "mean_device_ms": 1e3 * float(np.mean([t["done"] - t["launched"] for t in tm])),
            "mean_batch": float(np.mean([t["batch_size"] for t in tm])), "modes_not_ok_requests": bad,
            "max_batch": max_batch, "streams": n_streams}


def pct(a, q):
    return float(np.percentile(np.asarray(a), q))


def cpu_baseline(wl, every: int = 1):
    """The oracle as it stands on a bounded sample of the same workload:
    every `every`-th mode, all output times and multipoles; scaled to one
    full spectrum."""
    import oracle as O
    idx = np.arange(0, len(wl.k), every)
    t0 = time.perf_counter()
    t = O.build_tables(wl.cosmo, wl.prec, wl.k, wl.n_tau)
    S, st, ns, na = O.perturb(t, idx)
    DT, DE = O.los(t, S, wl.ell_max, True, k=t.k[idx])
    O.cl(t.k[idx], DT, DE, wl.ell_max, True, wl.cosmo["A_s"], wl.cosmo["n_s"])
    dt = time.perf_counter() - t0
    scale = len(wl.k) / len(idx)
    sec_per_spectrum = dt * scale
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": 1.0 / sec_per_spectrum, "unit": "spectra/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus_visible": os.cpu_count(),
            "sample": f"one fiducial spectrum: {len(idx)} of {len(wl.k)} modes, all {wl.n_tau} output times, "
                      f"l<=2500 (tables, perturbations, projection, quadrature); {dt:.1f} s measured"
                      + (f", scaled x{scale:.0f}" if every > 1 else "")}


def config2_sweep(ctx, batches):
    """Config 2 (config 1 plus one 0.06 eV neutrino: 12 momentum nodes with
    l <= 17, N = 295 rows, 600 modes): K1, K2, K3 of one batch timed with
    HIP events (median of the timed repeats after one untimed) and the
    spectra/s they give, per batch size."""
    import cmb_workloads as W
    import paper_2602_15104_amd as L
    import torch
    wl = W.config2()
    rows = []
    for B in batches:
        cosmos = W.perturbed_cosmologies(B, seed=20260215)
        for c in cosmos:
            for key in ("N_nu_massless", "Neff", "N_nu_massive", "m_nu_massive"):
                if key in wl.cosmo:
                    c[key] = wl.cosmo[key]
        t0 = time.perf_counter()
        tabs = [L.Tables(c, wl.prec, wl.k, wl.n_tau) for c in cosmos]
        t_tab = (time.perf_counter() - t0) / B
        n_k = len(wl.k)
        S = torch.empty((B, n_k, 3, wl.n_tau), dtype=torch.float64, device="cuda:0")
        st = torch.empty((B, n_k), dtype=torch.int32, device="cuda:0")
        D = torch.empty((B, 2, n_k, wl.ell_max - 1), dtype=torch.float64, device="cuda:0")
        C = torch.empty((B, 3, wl.ell_max + 1), dtype=torch.float64, device="cuda:0")
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        res = []
        for r in range(3):
            ev[0].record()
            ctx.perturb(tabs, S, st)
            ev[1].record()
            ctx.los(tabs, wl.ell_max, S, D)
            ev[2].record()
            ctx.cl(tabs, wl.ell_max, D, C)
            ev[3].record()
            torch.cuda.synchronize()
            res.append([ev[i].elapsed_time(ev[i + 1]) for i in range(3)])
        k1, k2, k3 = (float(v) for v in np.median(np.array(res[1:]), axis=0))
        rows.append({"batch": B, "spectra_per_s": 1000.0 * B / (k1 + k2 + k3), "perturb_ms": k1, "los_ms": k2,
                     "cl_ms": k3, "host_table_ms_per_cosmology": 1000.0 * t_tab,
                     "modes_not_ok": int((st != 0).sum().item())})
        print(f"[bench] config 2, batch {B}: {rows[-1]['spectra_per_s']:.1f} spectra/s", file=sys.stderr, flush=True)
        del S, st, D, C, tabs
    return {"workload": "config 1 + one 0.06 eV neutrino (12 momentum nodes, l <= 17), N = 295 rows, 600 modes, "
                        "2000 output times, l <= 2500", "rows": rows}


def gradient_only(args, W, L, dev):
    """The differentiation workload alone: cmb_gradient over a batch of
    config-1 cosmologies with seeded dL/dC_l, timed per call (host table
    builds of the perturbed cosmologies included)."""
    import torch
    wl = W.config1()
    B = args.batch
    cosmos = W.perturbed_cosmologies(B, seed=20260215)
    for c in cosmos:
        c["N_nu_massless"] = 3.0
    tabs = [L.Tables(c, wl.prec, wl.k, wl.n_tau) for c in cosmos]
    ctx = L.Context(0)
    lmax, n_k = wl.ell_max, len(wl.k)
    gen = torch.Generator(device="cpu").manual_seed(61)
    gC = torch.randn((B, 3, lmax + 1), generator=gen, dtype=torch.float64).to(dev)
    Gc = torch.empty((B, 3, lmax + 1), dtype=torch.float64, device=dev)
    Gg = torch.empty((B, 6), dtype=torch.float64, device=dev)
    Gs = torch.empty((B, n_k), dtype=torch.int32, device=dev)
    times = []
    for i in range(args.gradient_only):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.gradient(tabs, lmax, gC, Gc, Gg, Gs, rel=1e-4)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        print(f"[bench] gradient {i + 1}/{args.gradient_only}: {times[-1]:.3f} s", file=sys.stderr, flush=True)
    print(json.dumps({"metric": "dL/dtheta of C_ell (6 parameters) per second, batched", "value": B / min(times),
                      "unit": "gradients/s", "s_per_batch": min(times), "batch": B, "calls": len(times),
                      "modes_not_ok": int((Gs != 0).sum().item()), "dtype": "f64", "data": "synthetic",
                      "config": {"workload": "config-1 physics, batch of seeded cosmologies, seeded dL/dC_l, "
                                             "checkpoints every 64 steps"}}))
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--plain-reps", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variants", type=int, default=1, help="time the spectrum-side variants (0 = skip)")
    ap.add_argument("--serving-requests", type=int, default=512,
                    help="Poisson serving workload: requests replayed (0 = skip)")
    ap.add_argument("--serving-plain-requests", type=int, default=128,
                    help="the same arrivals served one request at a time (0 = skip)")
    ap.add_argument("--config2", type=str, default="",
                    help="also time config 2 (massive neutrino) at these comma-separated batch sizes")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration) and exit")
    ap.add_argument("--gradient-only", type=int, default=0, metavar="REPS",
                    help="only time the differentiation workload (config-1 physics, --batch cosmologies, "
                         "cmb_gradient) REPS times, print one JSON line and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path shards by cosmology "
              f"with no communication", file=sys.stderr)
        sys.exit(2)

    import torch
    import cmb_workloads as W
    import paper_2602_15104_amd as L

    assert torch.cuda.is_available(), "no GPU"
    dev = "cuda:0"
    if args.copy_calibration:
        n = 1 << 27  # 2^27 doubles = 1 GiB read + 1 GiB written per copy
        a = torch.ones(n, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n, "copies": 3}))
        return
    if args.gradient_only:
        gradient_only(args, W, L, dev)
        return
    wl = W.config1()
    B = args.batch
    cosmos = W.perturbed_cosmologies(B, seed=20260215)
    for c in cosmos:
        c["N_nu_massless"] = 3.0
    t0 = time.perf_counter()
    tabs = [L.Tables(c, wl.prec, wl.k, wl.n_tau) for c in cosmos]
    t_tables = (time.perf_counter() - t0) / B
    print(f"[bench] built {B} tables ({t_tables * 1e3:.1f} ms each)", file=sys.stderr, flush=True)
    ctx = L.Context(0)
    n_k, n_tau, lmax = len(wl.k), wl.n_tau, wl.ell_max
    N = 3 + (wl.prec["ell_gamma"] + 2) + (wl.prec["ell_pol"] + 1) + (wl.prec["ell_nu"] + 1)

    def alloc(b):
        return (torch.empty((b, n_k, 3, n_tau), dtype=torch.float64, device=dev),
                torch.empty((b, 2, n_k, lmax - 1), dtype=torch.float64, device=dev),
                torch.empty((b, 3, lmax + 1), dtype=torch.float64, device=dev),
                torch.empty((b, n_k), dtype=torch.int32, device=dev),
                torch.empty((b, n_k), dtype=torch.int32, device=dev))

    S, D, C, st, ns = alloc(B)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]

    def step(tb, bufs, times=None):
        S_, D_, C_, st_, ns_ = bufs
        ev[0].record()
        ctx.perturb(tb, S_, st_, ns_)
        ev[1].record()
        ctx.los(tb, lmax, S_, D_)
        ev[2].record()
        ctx.cl(tb, lmax, D_, C_)
        ev[3].record()
        if times is not None:
            times.append(ev)

    bufs = (S, D, C, st, ns)
    for i in range(args.warmup):
        step(tabs, bufs)
        torch.cuda.synchronize()
        print(f"[bench] warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    # timed batched steps
    kt = {"perturb": [], "los": [], "cl": []}
    step_ms = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        step(tabs, bufs)
        torch.cuda.synchronize()
        step_ms.append((time.perf_counter() - ts) * 1e3)
        kt["perturb"].append(ev[0].elapsed_time(ev[1]))
        kt["los"].append(ev[1].elapsed_time(ev[2]))
        kt["cl"].append(ev[2].elapsed_time(ev[3]))
        print(f"[bench] step {i + 1}/{args.steps}: {step_ms[-1]:.1f} ms", file=sys.stderr, flush=True)
    total = time.perf_counter() - t_start
    ms_per_step = total / args.steps * 1e3
    value = B * args.steps / total
    nsteps = ns.cpu().numpy()
    status = st.cpu().numpy()

    # plain: one cosmology per call, back to back
    pb = alloc(1)
    plain_ms = []
    for r in range(args.plain_reps + 1):
        ts = time.perf_counter()
        step([tabs[r % B]], pb)
        torch.cuda.synchronize()
        if r > 0:
            plain_ms.append((time.perf_counter() - ts) * 1e3)
    print(f"[bench] plain p50 {pct(plain_ms, 50):.1f} ms", file=sys.stderr, flush=True)

    # spectrum-side variants on the same batch (outside `value`): the transfer
    # k-grid (spline interpolation + projection + quadrature on 1699 points) and
    # the perturbation launch with the matter power spectrum today
    variants = {}
    if args.variants:
        ktg = L.transfer_kgrid(lmax, float(wl.k[0]), float(wl.k[-1]))
        St = torch.empty((B, len(ktg), 3, n_tau), dtype=torch.float64, device=dev)
        Dt = torch.empty((B, 2, len(ktg), lmax - 1), dtype=torch.float64, device=dev)
        Ct = torch.empty((B, 3, lmax + 1), dtype=torch.float64, device=dev)
        Pk = torch.empty((B, n_k), dtype=torch.float64, device=dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        tg, tp = [], []
        for r in range(3):
            e0.record()
            ctx.spectra_on_grid(tabs, lmax, S, ktg, St, Dt, Ct)
            e1.record()
            torch.cuda.synchronize()
            tg.append(e0.elapsed_time(e1))
            e0.record()
            ctx.perturb_pk(tabs, S, st, Pk, ns)
            e1.record()
            torch.cuda.synchronize()
            tp.append(e0.elapsed_time(e1))
        variants["transfer_grid"] = {"n_kt": len(ktg), "ms_per_batch": float(np.median(tg[1:])),
                                     "batch": B, "what": "natural-spline sources onto the App. A.2 transfer grid, "
                                                         "projection and k quadrature there"}
        variants["perturb_pk"] = {"ms_per_batch": float(np.median(tp[1:])), "batch": B,
                                  "perturb_ms": float(np.mean(kt["perturb"]))}
        del St, Dt, Ct, Pk
        # three-region Bessel scheme in the projection (table built outside the timing)
        D3 = torch.empty_like(D)
        t0b = time.perf_counter()
        ctx.los_bessel3(tabs[:1], lmax, S[:1], D3[:1])
        torch.cuda.synchronize()
        t_b3 = time.perf_counter() - t0b
        t3 = []
        for r in range(3):
            e0.record()
            ctx.los_bessel3(tabs, lmax, S, D3)
            e1.record()
            torch.cuda.synchronize()
            t3.append(e0.elapsed_time(e1))
        variants["los_bessel3"] = {"ms_per_batch": float(np.median(t3[1:])), "los_ms": float(np.mean(kt["los"])),
                                   "first_call_s_incl_table": t_b3, "batch": B}
        del D3
        # lensing: K1 with delta_m at the output times, the Limber potential
        # spectrum, and lensed TT/TE/EE/BB (l <= 2000 from l <= 2500, 3700 nodes)
        Dm = torch.empty((B, n_k, n_tau), dtype=torch.float64, device=dev)
        Pp = torch.empty((B, lmax + 1), dtype=torch.float64, device=dev)
        l_out, n_mu = 2000, 3700
        Cll = torch.empty((B, 4, l_out + 1), dtype=torch.float64, device=dev)
        ctx.lensed_cl(C, Pp.zero_(), l_out, Cll, n_mu=n_mu)  # node tables outside the timing
        torch.cuda.synchronize()
        e2 = torch.cuda.Event(enable_timing=True)
        tm, tl, tz = [], [], []
        for r in range(3):
            e0.record()
            ctx.perturb_matter(tabs, S, st, Dm=Dm, nsteps=ns)
            e1.record()
            ctx.lensing_potential(tabs, lmax, Dm, Pp)
            e2.record()
            torch.cuda.synchronize()
            tm.append(e0.elapsed_time(e1))
            tl.append(e1.elapsed_time(e2))
            e0.record()
            ctx.lensed_cl(C, Pp, l_out, Cll, n_mu=n_mu)
            e1.record()
            torch.cuda.synchronize()
            tz.append(e0.elapsed_time(e1))
        variants["lensing"] = {"perturb_with_delta_m_ms": float(np.median(tm[1:])),
                               "limber_ms": float(np.median(tl[1:])), "lensed_cl_ms": float(np.median(tz[1:])),
                               "lensed_l_max": l_out, "unlensed_l_max": lmax, "n_mu": n_mu, "batch": B}
        del Dm, Pp, Cll
        # reverse mode of the spectrum side: dL/dS from dL/dC_l (transposed k
        # quadrature and projection) for the batch, at the batch's Delta
        gCl = torch.ones((B, 3, lmax + 1), dtype=torch.float64, device=dev)
        gS = torch.empty_like(S)
        ta = []
        for r in range(3):
            e0.record()
            ctx.spectra_adjoint(tabs, lmax, D, gCl, gS)
            e1.record()
            torch.cuda.synchronize()
            ta.append(e0.elapsed_time(e1))
        variants["spectra_adjoint"] = {"ms_per_batch": float(np.median(ta[1:])), "batch": B,
                                       "los_ms": float(np.mean(kt["los"]))}
        # transposed source functions for one cosmology (dL/dy at every output
        # time and state row: n_k n_tau rows doubles written)
        rows = tabs[0].state_rows()
        gY = torch.empty((1, n_k, n_tau, rows), dtype=torch.float64, device=dev)
        tsa = []
        for r in range(3):
            e0.record()
            ctx.sources_adjoint(tabs[:1], gS[:1], gY)
            e1.record()
            torch.cuda.synchronize()
            tsa.append(e0.elapsed_time(e1))
        t_sa = float(np.median(tsa[1:]))
        by = 8.0 * n_k * n_tau * (rows + 3)
        variants["sources_adjoint"] = {"ms_per_cosmology": t_sa, "bytes": by, "GB_per_s": by / (t_sa * 1e6),
                                       "rows": rows}
        del gCl, gS, gY
        # trajectory checkpoints every 64 accepted steps: the batch's recorded
        # steps replayed plain, replayed writing the checkpoints, and every
        # segment replayed from its checkpoint (the forward recomputation of a
        # checkpointed reverse sweep), into one source buffer
        every = 64
        cap = int(wl.prec["max_steps"]) + 1
        Hh = torch.empty((B, n_k, cap), dtype=torch.float64, device=dev)
        Hn = torch.empty((B, n_k), dtype=torch.int32, device=dev)
        ctx.perturb_record(tabs, S, st, Hh, Hn)
        ck = torch.empty((B, n_k, (cap - 1) // every + 1, 1 + 2 * rows), dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        n_seg = int(Hn.max().item()) // every + 1
        e2 = torch.cuda.Event(enable_timing=True)
        e3 = torch.cuda.Event(enable_timing=True)
        trp, tck, tsg = [], [], []
        for r in range(3):
            e0.record()
            ctx.perturb_replay(tabs, Hh, Hn, S, st)
            e1.record()
            ctx.perturb_checkpoint(tabs, Hh, Hn, every, ck, S, st, replay=True)
            e2.record()
            for sg in range(n_seg):
                ctx.perturb_segment(tabs, Hh, Hn, every, ck, sg, S, st)
            e3.record()
            torch.cuda.synchronize()
            trp.append(e0.elapsed_time(e1))
            tck.append(e1.elapsed_time(e2))
            tsg.append(e2.elapsed_time(e3))
        used = float(((Hn.to(torch.float64) // every) + 1).sum().item()) * (1 + 2 * rows) * 8.0
        variants["checkpoints"] = {"every": every, "replay_ms": float(np.median(trp[1:])),
                                   "replay_with_checkpoints_ms": float(np.median(tck[1:])),
                                   "all_segments_ms": float(np.median(tsg[1:])), "segments": n_seg,
                                   "checkpoint_bytes_written": used, "checkpoint_buffer_bytes": ck.numel() * 8.0,
                                   "modes_not_ok": int((st != 0).sum().item()), "batch": B}
        del Hh, Hn, ck
        # parameter derivatives: C_l and dC_l/d(h, omega_b, omega_cdm, ln A_s, n_s,
        # tau_reio) for the batch (five-point frozen-step stencil, rel 1e-4;
        # host table builds of the perturbed cosmologies included)
        Jc = torch.empty((B, 3, lmax + 1), dtype=torch.float64, device=dev)
        Jj = torch.empty((B, 6, 3, lmax + 1), dtype=torch.float64, device=dev)
        Js = torch.empty((B, n_k), dtype=torch.int32, device=dev)
        torch.cuda.synchronize()
        tj0 = time.perf_counter()
        ctx.jacobian(tabs, lmax, Jc, Jj, Js, rel=1e-4, order=4)
        torch.cuda.synchronize()
        tj = time.perf_counter() - tj0
        variants["jacobian"] = {"s_per_batch": tj, "gradients_per_s": B / tj, "order": 4, "rel": 1e-4,
                                "cosmologies_integrated": B * 17, "batch": B,
                                "modes_not_ok": int((Js != 0).sum().item())}
        del Jc, Jj, Js
        # the discrete adjoint: C_l and dL/dtheta of L = sum gC C_l for seeded
        # gC (record with checkpoints, spectrum-side reverse mode, segment
        # replays and the reverse ESDIRK sweep, table tangents; host table
        # builds of the perturbed cosmologies included)
        gen = torch.Generator(device="cpu").manual_seed(61)
        gC = torch.randn((B, 3, lmax + 1), generator=gen, dtype=torch.float64).to(dev)
        Gc = torch.empty((B, 3, lmax + 1), dtype=torch.float64, device=dev)
        Gg = torch.empty((B, 6), dtype=torch.float64, device=dev)
        Gs = torch.empty((B, n_k), dtype=torch.int32, device=dev)
        tgs = []
        for _ in range(2):
            torch.cuda.synchronize()
            tg0 = time.perf_counter()
            ctx.gradient(tabs, lmax, gC, Gc, Gg, Gs, rel=1e-4)
            torch.cuda.synchronize()
            tgs.append(time.perf_counter() - tg0)
        tg = min(tgs)
        variants["gradient"] = {"s_per_batch": tg, "gradients_per_s": B / tg, "rel": 1e-4, "batch": B,
                                "jacobian_over_adjoint_time": tj / tg, "modes_not_ok": int((Gs != 0).sum().item()),
                                "what": "cmb_gradient: record + checkpoints, spectrum-side adjoint, per 64-step "
                                        "segment a replay and the reverse ESDIRK sweep, table tangents"}
        del gC, Gc, Gg, Gs
        print(f"[bench] variants: transfer grid {variants['transfer_grid']['ms_per_batch']:.1f} ms, "
              f"perturb+pk {variants['perturb_pk']['ms_per_batch']:.1f} ms, "
              f"los three-region {variants['los_bessel3']['ms_per_batch']:.1f} ms, lensing "
              f"{variants['lensing']}, spectra adjoint {variants['spectra_adjoint']['ms_per_batch']:.1f} ms, "
              f"sources adjoint {variants['sources_adjoint']['ms_per_cosmology']:.2f} ms per cosmology, "
              f"checkpoints {variants['checkpoints']}, jacobian {variants['jacobian']['s_per_batch']:.2f} s, "
              f"adjoint gradient {variants['gradient']['s_per_batch']:.2f} s",
              file=sys.stderr, flush=True)

    # roofline of the dominant kernel (algorithmic flops / measured duration):
    # the perturbation kernel on the scope's count of 560 N per step (the
    # reported fraction), and beside it on the count of what this kernel's
    # continuant solve executes (fewer operations for the same solution)
    exs = [t.export() for t in tabs]
    f_k1 = float(np.sum(nsteps)) * k1_flops_per_step_scope(N)
    f_k1_exec = float(np.sum(nsteps)) * k1_flops_per_step(N) + B * n_k * n_tau * K1_FLOPS_PER_OUTPUT
    f_k2 = sum(k2_flops(e["k"], e["chi_src"], lmax) for e in exs)
    f_k3 = 12.0 * B * (lmax - 1) * n_k
    avg = {k: float(np.mean(v)) for k, v in kt.items()}
    flops = {"perturb": f_k1, "los": f_k2, "cl": f_k3}
    dom = max(avg, key=avg.get)
    achieved = flops[dom] / (avg[dom] * 1e-3) / 1e12
    per_kernel = {k: {"ms": avg[k], "tflops": flops[k] / (avg[k] * 1e-3) / 1e12,
                      "frac_fp64_peak": flops[k] / (avg[k] * 1e-3) / 1e12 / FP64_PEAK_TFLOPS} for k in avg}
    per_kernel["perturb"]["count"] = "560 N flops per ESDIRK step (banded LU + Woodbury stage solve), N = %d" % N
    per_kernel["perturb"]["tflops_executed_count"] = f_k1_exec / (avg["perturb"] * 1e-3) / 1e12
    per_kernel["perturb"]["frac_executed_count"] = per_kernel["perturb"]["tflops_executed_count"] / FP64_PEAK_TFLOPS
    per_kernel["perturb"]["executed_count"] = ("%.0f flops per step (continuant stage solve as executed) + %.0f per "
                                               "output time" % (k1_flops_per_step(N), K1_FLOPS_PER_OUTPUT))
    fp64_meas = k_fp64_measured(B)
    if fp64_meas:
        for k, v in fp64_meas.items():
            if k in per_kernel:
                per_kernel[k]["tflops_counters"] = v["flops_per_launch"] / (avg[k] * 1e-3) / 1e12
                per_kernel[k]["counters"] = v["what"]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "spectra/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "TT/TE/EE ell<=2500, 400 k (log/linear step law 1e-5..0.5 Mpc^-1), 2000 output "
                               "times, photon T+P and massless-nu hierarchies to l=24, batched cosmologies "
                               "(5% Gaussian around LCDM fiducial)",
                   "batch": B, "n_k": n_k, "n_tau": n_tau, "ell_max": lmax, "state_rows": N},
        "batched": {"spectra_per_s": value, "step_ms_p50": pct(step_ms, 50), "step_ms_p99": pct(step_ms, 99)},
        "plain": {"spectra_per_s": 1e3 / pct(plain_ms, 50), "p50_ms": pct(plain_ms, 50),
                  "p99_ms": pct(plain_ms, 99), "reps": len(plain_ms)},
        "batched_over_plain": value / (1e3 / pct(plain_ms, 50)),
        "kernels": per_kernel,
        "mean_steps_per_mode": float(np.mean(nsteps)),
        "modes_not_ok": int(np.sum(status != 0)),
        "host_table_ms_per_cosmology": t_tables * 1e3,
        "variants": variants,
        "roofline": {"bound": "alu", "kernel": dom, "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": k1_traffic(B) if dom == "perturb" else None,
                     "count": per_kernel[dom].get("count", "algorithmic flops of the kernel"),
                     "frac_executed_count": per_kernel[dom].get("frac_executed_count"),
                     "achieved_counters": per_kernel[dom].get("tflops_counters")},
    }
    if args.serving_requests > 0:
        reqs = W.serving_requests(args.serving_requests, rate_hz=50.0, seed=20260215)
        print(f"[bench] serving {len(reqs)} Poisson requests (50/s)", file=sys.stderr, flush=True)
        out["serving"] = serve(reqs, wl.prec, wl.n_tau, max_batch=64, n_streams=2)
        out["serving"]["workload"] = ("512 requests, Poisson 50/s, 5% Gaussian cosmologies, l_max in {500, 1000, "
                                      "2500} with 100/250/400 modes on [1e-5, 0.5 l_max/2500], 2000 output times, "
                                      "config-1 hierarchy; latency = arrival to spectra on the host, incl. host tables")
        print(f"[bench] serving p50 {out['serving']['p50_ms']:.1f} ms p99 {out['serving']['p99_ms']:.1f} ms",
              file=sys.stderr, flush=True)
        # capacity: the same requests arriving 40 times faster (2000/s), so the
        # runtime is saturated and throughput is what it can serve
        fast = [dict(r, arrival_s=r["arrival_s"] / 40.0) for r in reqs]
        out["serving_saturated"] = serve(fast, wl.prec, wl.n_tau, max_batch=64, n_streams=2)
        out["serving_saturated"]["workload"] = "the same 512 requests, arrivals compressed 40x (2000/s offered)"
        print(f"[bench] serving saturated: {out['serving_saturated']['throughput_per_s']:.1f} requests/s, "
              f"p50 {out['serving_saturated']['p50_ms']:.1f} ms", file=sys.stderr, flush=True)
        if args.serving_plain_requests > 0:
            sub = reqs[:args.serving_plain_requests]
            out["serving_plain"] = serve(sub, wl.prec, wl.n_tau, max_batch=1, n_streams=1)
            print(f"[bench] serving one-at-a-time p50 {out['serving_plain']['p50_ms']:.1f} ms", file=sys.stderr,
                  flush=True)
    if args.config2:
        out["config2"] = config2_sweep(ctx, [int(b) for b in args.config2.split(",")])
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle sample)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
