"""Throughput of the batched likelihood evaluation on one MI355X.

Workload: the Fabry-Perot-like galaxy, 128 x 128 spatial x 48 channels of
16 km/s, exponential disc r0 = 20 px, exponential-rise rotation curve,
PSF FWHM 3 px, LSF FWHM 30 km/s, noise 3 km/s, flux mask at 1% of the peak.
One step = one batched evaluation (model cube -> PSF/LSF -> moments ->
masked chi-square) of 400 parameter rows, the live-point batch of the nested
sampler, drawn from the workload's generative ranges; every step uses a
different batch, all resident in device memory before timing starts.

Prints one JSON line: evals/s, the roofline of the dominant kernel (timed
live with HIP events on the launch stream) and the CPU oracle baseline, plus
fits/hour of the surrogate workload (64 x 64 x 64 instrument): the network
trained on 2 M rows streamed from the plain evaluation, then nested-sampling
fits (1000 live points, 10 free parameters) of synthetic galaxies, plain and
surrogate-screened, with the posterior medians compared; and the
velocity-field strategy (Sec. 2.2.1) on GHASP-shaped 256^2 and 512^2 maps:
evals/s of 1024-row launches, its kernel's roofline, LM and nested-sampling
fits, Monte-Carlo errors and the oracle's rate; the survey-shaped and 700^2
cubes; and Gaussian line fitting of 262,144 spectra.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "model evals/s (cube+PSF+moments+χ²); fits/hour, surrogate vs plain"
BATCH = 400

# MI355X FP64 vector peak: 256 CUs x 64 lanes x 2.4 GHz x 2 FLOP (FMA)
# = 78.6 TFLOP/s.  The dominant kernel, k_line_sums, runs its per-voxel work in
# FP64; packed FP32 is not used anywhere.
LANE_OPS_PER_S = 256 * 64 * 2.4e9
PEAK_TFLOPS = 2 * LANE_OPS_PER_S / 1e12
# Algorithmic work of k_line_sums.  Per fine spaxel of the halo-extended grid
# (every row): eqs. 1-8 and the line's start values.  FP64 FLOP of the FP64
# parts (FMA = 2): x_e and y_e/cos i (4 FMA = 8), r^2 (MUL + FMA = 3), the
# Newton step of 1/r (3 MUL + FMA = 5), r (1), the brightness exponent
# (MUL + FMA = 3), Vsys + projected rotation (1), the line centre in channels
# (ADD + MUL = 2), the first channel's offset (ADD + MUL = 2), the two
# recurrence start arguments (FMA; FMA + MUL = 5) and their fractional parts
# (2 ADD): 32.  VALU issue slots: ~40 operations and 3 transcendentals
# (the rotation curve's atan or exp, the two start exp2) at 4 slots each: 52.
# Per line-support voxel: the profile by the ratio recurrence (g *= r,
# r *= q) and three weighted sums (3 FMA): 8 FP64 FLOP in 5 slots.
SPAXEL_FLOP, SPAXEL_SLOTS = 32, 52
FLOP_PER_VOXEL, VOXEL_SLOTS = 8, 5
PEAK_HBM_GBS = 8000.0
PEAK_BF16_TFLOPS = 2500.0  # dense BF16 MFMA, published (no 2:1 sparsity)

# HBM traffic per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
# passes; reported only while the kernel sources still hash to the profiled ones
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_c2_128x128x48.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1510_01815_amd", "csrc", f)
                  for f in ("gbk_kernels.hip", "gbk_internal.h")]


TIME_EVERY = 10  # one step in TIME_EVERY of the timed region is timed kernel by kernel
# acceptances per nested-sampling round (adaptive batch) of the surrogate
# workload's fits, plain and screened alike: N/5 for N = 1000 live points
ACCEPT_TARGET = 200
# the screened fits screen a round only where it pays: a surrogate row costs
# ~0.24 plain rows on the 64x64x64 instrument and the screen ~500 plain rows per
# round (measured on MI355X); 0.3 and 300 fitted best over the six galaxies
SCREEN_COST, SCREEN_ROWS = 0.3, 300
FIT_CAP_S = 8.0  # wall-time cap of one nested-sampling fit of the surrogate workload

# Velocity-field strategy (Sec. 2.2.1) on GHASP-shaped maps: batch of the
# timed launches, and the kernel's executed FP64 FLOP and VALU instructions per
# pixel on the Epinat curve, from the SQ_INSTS_VALU_{FMA,ADD,MUL,TRANS}_F64 and
# SQ_INSTS_VALU counters of the 512 x 512 x 1024-row launches (FMA = 2 FLOP; the
# FP64 elementary functions' polynomial evaluations included)
VF_BATCH = 1024
MC_SIMS = 200  # simulated velocity fields per galaxy for the Monte-Carlo errors (Sec. 4.2)
VF_FLOP_PER_PIXEL = 170.3
VF_VALU_PER_PIXEL = 187.1
# wave64 VALU issue peak: 256 CUs x 4 SIMDs x 2.4 GHz, one wave instruction per 4 cycles
VALU_ISSUE_PER_S = 256 * 4 * 2.4e9 / 4


def kernel_source_hash() -> str:
    """SHA-256 of the kernel sources' code: // comments, trailing blanks and
    blank lines are dropped, so that edits to comments keep the counters valid."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, encoding="utf-8") as fh:
            for line in fh:
                code = re.sub(r"//.*", "", line).rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()


def measured_counters() -> dict:
    """{kernel: {"hbm_bytes": HBM bytes per launch, "SQ_INSTS_VALU": wave
    instructions per launch}} from the committed counter summary, or {} when
    the kernel sources no longer hash to the profiled ones."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return {}
    if t.get("source_sha256") != kernel_source_hash():
        return {}
    out = {}
    for k, v in t["kernels"].items():
        out[k] = {"hbm_bytes": round(v["FETCH_SIZE_KiB"] * 1024 * t["fetch_factor"] +
                                     v["WRITE_SIZE_KiB"] * 1024 * t["write_factor"])}
        if "SQ_INSTS_VALU" in v:
            out[k]["SQ_INSTS_VALU"] = v["SQ_INSTS_VALU"]
    return out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows-per-thread", type=int, default=12,
                    help="oracle rows per thread of each all-core run")
    ap.add_argument("--cpu-rows-single", type=int, default=40,
                    help="oracle rows of each one-core run")
    ap.add_argument("--fit-galaxies", type=int, default=6,
                    help="galaxies of the surrogate workload fitted both ways (0: skip)")
    ap.add_argument("--train-rows", type=int, default=2_000_000)
    ap.add_argument("--surrogate-kernels-only", action="store_true",
                    help="time only the surrogate's GEMM and screening pass (for counter runs)")
    ap.add_argument("--survey-galaxies", type=int, default=2000,
                    help="galaxies of the uneven-survey LM workload (0: skip)")
    ap.add_argument("--grid-galaxies", type=int, default=10,
                    help="galaxies of the nested-grid workload (0: skip)")
    ap.add_argument("--ns-fits", type=int, default=3,
                    help="nested-sampling fits of the 128x128x48 workload (0: skip)")
    ap.add_argument("--no-line-fit", action="store_true", help="skip the line-fitting workload")
    ap.add_argument("--no-large-cubes", action="store_true", help="skip the survey/high-res shapes")
    ap.add_argument("--vfield-galaxies", type=int, default=4,
                    help="LM fits of the velocity-field workload (-1: skip the workload)")
    return ap.parse_args()


def other_workloads(gbk, I, torch, n_survey, n_grid, n_ns, precision_samples):
    """Fits/hour and evals/s of the other optimiser workloads (subsets, labelled).
    Appends (grid, rows, GPU maps) of sampled nested-grid nodes to
    precision_samples for the oracle comparison of the CPU leg."""
    dev = torch.device("cuda:0")
    out = {}
    if n_ns > 0:
        # the Fabry-Perot workload fitted by nested sampling: 400 live points, the
        # 10 non-Epinat parameters, every round's candidates in one launch
        grid = I.c2_grid()
        lo, hi = I.c2_prior_box()
        ts, ev, ln, cov = [], [], [], []
        for k in range(n_ns):
            truth = I.c2_draw(I.rng_for(2, 10 + k, 40), 1)[0]
            mk = gbk.Model.from_grid(grid)
            mp = mk.evaluate(torch.tensor(truth[None], device=dev)).cpu().numpy()[0]
            mk.set_obs(I.make_observation(mp, 3.0, I.rng_for(2, 10 + k, 41)))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = mk.fit_nested(lo, hi, [1] * 10 + [0, 0], truth, n_live=400, seed=k + 1)
            ts.append(time.perf_counter() - t0)
            ev.append(r["n_evals"])
            ln.append(r["n_launches"])
            cov.append(int(np.sum((r["q16"][:10] <= truth[:10]) & (truth[:10] <= r["q84"][:10]))))
            log(f"128x128x48 nested sampling fit {k}: {ts[-1]:.2f} s, {r['n_evals']} evaluations")
        out["ns_128x128x48"] = {"fits": n_ns, "n_live": 400, "free": 10,
                                "s_per_fit": round(float(np.mean(ts)), 4),
                                "fits_per_hour": round(3600 * n_ns / sum(ts), 1),
                                "evals_per_fit": float(np.mean(ev)),
                                "launches_per_fit": float(np.mean(ln)),
                                "evals_per_s": round(sum(ev) / sum(ts), 1),
                                "truth_in_68pct_of_10": cov}
    free9 = [1, 1, 1, 1, 1, 1, 1, 1, 1, 0, 0, 0]
    # single galaxy, 32x32x64, plain LM from a 20% perturbed start
    m = gbk.Model.from_grid(I.c1_grid())
    truth = I.c1_truth()
    maps = m.evaluate(torch.tensor(truth[None], device=dev)).cpu().numpy()[0]
    m.set_obs(I.make_observation(maps, 5.0, I.rng_for(1, 0, 1)))
    ts, evals = [], []
    for k in range(5):
        t0 = time.perf_counter()
        r = m.fit_lm(I.c1_start(I.rng_for(1, k, 2)), free9)
        ts.append(time.perf_counter() - t0)
        evals.append(r["n_evals"])
    log("single-galaxy LM fits done")
    out["lm_32x32x64"] = {"fits": 5, "fits_per_hour": round(3600 * 5 / sum(ts), 1),
                          "evals_per_fit": float(np.mean(evals)),
                          "evals_per_s": round(sum(evals) / sum(ts), 1)}
    if n_survey > 0:
        gals = I.c3_survey(n_survey)
        models, p0 = [], []
        for k, g in enumerate(gals):
            mk = gbk.Model.from_grid(g.grid)
            mp = mk.evaluate(torch.tensor(g.truth[None], device=dev)).cpu().numpy()[0]
            mk.set_obs(I.make_observation(mp, g.noise, I.rng_for(3, k, 1), random_mask=0.1))
            models.append(mk)
            rng = I.rng_for(3, k, 2)
            start = g.truth.copy()
            for s_ in range(9):
                sign = 1.0 if rng.random() < 0.5 else -1.0
                start[s_] = start[s_] + sign * 6.0 if s_ == I.VSYS else start[s_] * (1.0 + 0.2 * sign)
            p0.append(start)
        log(f"survey of {n_survey} galaxies set up")
        sv = gbk.Survey(models)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = sv.fit_lm(np.array(p0), free9)
        dt = time.perf_counter() - t0
        log(f"survey LM done in {dt:.2f} s")
        out["survey_lm"] = {"galaxies": n_survey, "of": 2000, "capped": int(np.sum(np.array(r["reason"]) == "maxiter")),
                            "fits_per_hour": round(3600 * n_survey / dt, 1),
                            "seconds": round(dt, 3), "evals": int(r["n_evals"].sum()),
                            "evals_per_s": round(float(r["n_evals"].sum()) / dt, 1),
                            "mean_iterations": float(np.mean(r["iterations"]))}
        sv.close()
    if n_grid > 0:
        ts, ev = [], 0
        for k in range(n_grid):
            g, truth = I.c4_galaxy(k)
            mg = gbk.Model.from_grid(g)
            mp = mg.evaluate(torch.tensor(truth[None], device=dev)).cpu().numpy()[0]
            mg.set_obs(I.make_observation(mp, 5.0, I.rng_for(4, k, 1)))
            lo, hi = truth.copy(), truth.copy()
            for slot, (a, b) in {I.INC: (5.0, 85.0), I.PA: (0.0, 360.0), I.VT: (50.0, 300.0),
                                 I.RT: (0.5 * g.psf_fwhm, 2.0 * g.psf_fwhm),
                                 I.SIG: (20.0, 100.0)}.items():
                lo[slot], hi[slot] = a, b
            free = [0] * 12
            for slot in (I.INC, I.PA, I.VT, I.RT, I.SIG):
                free[slot] = 1
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = mg.fit_grid(lo, hi, free, truth, n_per_dim=16, max_levels=3)
            ts.append(time.perf_counter() - t0)
            ev += r["n_evals"]
            # sampled nodes for the precision study: the best node and two nodes
            # of the first level's grid
            nodes = np.stack([r["best"]] * 3)
            rs = I.rng_for(4, k, 7)
            for j in (1, 2):
                for slot in (I.INC, I.PA, I.VT, I.RT, I.SIG):
                    nodes[j, slot] = lo[slot] + rs.integers(16) / 15.0 * (hi[slot] - lo[slot])
            gm = mg.evaluate(torch.tensor(nodes, device=dev)).cpu().numpy()
            precision_samples.append((g, nodes, gm))
            log(f"nested grid galaxy {k}: {ts[-1]:.2f} s")
        out["nested_grid_30x30x64"] = {"galaxies": n_grid, "of": 1000,
                                       "fits_per_hour": round(3600 * n_grid / sum(ts), 1),
                                       "evals_per_s": round(ev / sum(ts), 1),
                                       "evals_per_fit": ev / n_grid}
    return out


def velocity_field_workload(gbk, I, torch, n_fit, cpu):
    """The velocity-field strategy on GHASP-shaped maps (Epinat curve,
    velocity only): evals/s of 1024-row chi-square launches at 256^2 and 512^2,
    the kernel's roofline, LM fits of 512^2 galaxies, and the oracle's rate."""
    dev = torch.device("cuda:0")
    out = {"workload": "GHASP-shaped velocity fields (Fabry-Perot, Sec. 4.2): Epinat curve, "
                       "velocity only (W = 0), coverage to ~3 disc scale lengths with 30% holes, "
                       f"noise 5 km/s, {VF_BATCH} rows per launch"}
    for side in (256, 512):
        grid = I.ghasp_grid(side)
        m = gbk.Model.from_grid(grid)
        rows = I.ghasp_draw(I.rng_for(6, side, 0), 21 * VF_BATCH, side)
        mp = m.evaluate(torch.tensor(rows[:1], device=dev)).cpu().numpy()[0]
        m.set_obs(I.make_observation(mp, 5.0, I.rng_for(6, side, 1), flux_frac=I.GHASP_FLUX_FRAC,
                                     random_mask=I.GHASP_HOLES, W=0.0))
        batches = torch.tensor(rows.reshape(21, VF_BATCH, I.NPAR), device=dev)
        c2 = torch.empty((21, VF_BATCH), dtype=torch.float64, device=dev)
        nv = torch.empty((21, VF_BATCH), dtype=torch.int64, device=dev)
        stream = torch.cuda.current_stream()
        for k in range(3):
            m.chi2(batches[k], out=c2[k], n_valid=nv[k], stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(1, 21):
            m.chi2(batches[k], out=c2[k], n_valid=nv[k], stream=stream)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 20
        m.set_profiling(gbk.GK_PROF_TIMING)
        for k in range(1, 11):
            m.chi2(batches[k], out=c2[k], n_valid=nv[k], stream=stream)
        prof = m.read_profile()
        m.set_profiling(0)
        kms = prof["kernel_ms"]["k_line_sums"] / max(prof["launches"]["k_line_sums"], 1)
        px = VF_BATCH * side * side
        entry = {"evals_per_s": round(VF_BATCH / dt, 1), "ms_per_launch": round(1e3 * dt, 4),
                 "k_vfield_ms": round(kms, 5)}
        if side == 512:
            tf = px * VF_FLOP_PER_PIXEL / (kms * 1e-3) / 1e12
            issue = px * VF_VALU_PER_PIXEL / 64 / (kms * 1e-3)
            entry["roofline"] = {"bound": "alu", "kernel": "k_vfield", "achieved": round(tf, 3),
                                 "peak": round(PEAK_TFLOPS, 1), "unit": "TFLOP/s",
                                 "frac": round(tf / PEAK_TFLOPS, 4), "traffic": None,
                                 "flop_per_pixel": VF_FLOP_PER_PIXEL,
                                 "valu_issue_frac": round(issue / VALU_ISSUE_PER_S, 4)}
            assert np.isfinite(c2.cpu().numpy()).all()
        out[f"{side}x{side}"] = entry
        log(f"velocity field {side}^2: {VF_BATCH / dt:.0f} evals/s")
    if n_fit > 0:
        side = 512
        grid = I.ghasp_grid(side)
        lo, hi = I.ghasp_box(side)
        ts, ev, it = [], [], []
        for k in range(n_fit):
            truth = I.ghasp_draw(I.rng_for(6, 100 + k, 0), 1, side)[0]
            m = gbk.Model.from_grid(grid)
            mp = m.evaluate(torch.tensor(truth[None], device=dev)).cpu().numpy()[0]
            m.set_obs(I.make_observation(mp, 5.0, I.rng_for(6, 100 + k, 1),
                                         flux_frac=I.GHASP_FLUX_FRAC, random_mask=I.GHASP_HOLES,
                                         W=0.0))
            p0 = I.ghasp_start(I.rng_for(6, 100 + k, 2), truth, side)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = m.fit_lm(p0, I.GHASP_FREE, lo, hi)
            ts.append(time.perf_counter() - t0)
            ev.append(r["n_evals"])
            it.append(r["iterations"])
        out["lm_512x512"] = {"fits": n_fit, "free": 7, "s_per_fit": round(float(np.mean(ts)), 4),
                             "fits_per_hour": round(3600 * n_fit / sum(ts), 1),
                             "evals_per_fit": float(np.mean(ev)),
                             "iterations_per_fit": float(np.mean(it))}
        log(f"velocity-field LM fits: {np.mean(ts):.3f} s each")
        # nested sampling of the same galaxies (the paper's settings, Sec. 4: 50 live
        # points, tolerance 0.5), 7 free parameters in a box about the truth
        ts_ns, ev_ns = [], []
        for k in range(n_fit):
            truth = I.ghasp_draw(I.rng_for(6, 100 + k, 0), 1, side)[0]
            mk = gbk.Model.from_grid(grid)
            mp = mk.evaluate(torch.tensor(truth[None], device=dev)).cpu().numpy()[0]
            mk.set_obs(I.make_observation(mp, 5.0, I.rng_for(6, 100 + k, 1),
                                          flux_frac=I.GHASP_FLUX_FRAC, random_mask=I.GHASP_HOLES,
                                          W=0.0))
            blo, bhi = truth.copy(), truth.copy()
            for slot, w in ((I.PA, 20.0), (I.INC, 10.0), (I.VSYS, 30.0), (I.VT, 60.0),
                            (I.RT, 0.3 * truth[I.RT]), (I.A, 0.3), (I.G, 0.3)):
                blo[slot], bhi[slot] = truth[slot] - w, truth[slot] + w
            blo[I.INC], bhi[I.INC] = max(blo[I.INC], 5.0), min(bhi[I.INC], 85.0)
            blo[I.G] = max(blo[I.G], 0.05)
            blo[I.A] = max(blo[I.A], 0.0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rn = mk.fit_nested(blo, bhi, I.GHASP_FREE, truth, n_live=50, tol=0.5, seed=k + 1)
            ts_ns.append(time.perf_counter() - t0)
            ev_ns.append(rn["n_evals"])
        out["ns_512x512"] = {"fits": n_fit, "free": 7, "n_live": 50, "s_per_fit": round(float(np.mean(ts_ns)), 4),
                             "fits_per_hour": round(3600 * n_fit / sum(ts_ns), 1),
                             "evals_per_fit": float(np.mean(ev_ns))}
        log(f"velocity-field NS fits: {np.mean(ts_ns):.3f} s each")
        # Monte-Carlo errors of the last galaxy (Sec. 4.2): 200 shuffled residual
        # fields about its fit, refitted in batched groups
        best = r["p"]
        perm = I.mc_permutations(I.rng_for(6, 199, 3), MC_SIMS, m.n_valid())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mc = m.mc_errors(best, I.GHASP_FREE, lo, hi, "shuffle", perm=perm)
        dt = time.perf_counter() - t0
        out["mc_errors_512x512"] = {"simulations": MC_SIMS, "seconds": round(dt, 4),
                                    "refits_per_s": round(MC_SIMS / dt, 1),
                                    "galaxies_per_hour": round(3600 / dt, 1),
                                    "capped_fits": mc["n_capped"]}
        log(f"Monte-Carlo errors, {MC_SIMS} refits: {dt:.3f} s")
    if cpu:
        from concurrent.futures import ThreadPoolExecutor

        from oracle import oracle as O
        O.lib()
        side = 512
        d = O.Desc(side, side, 1, rc=I.RC_EPINAT)
        threads = host_threads()
        rows = I.ghasp_draw(I.rng_for(6, side, 0), 64 * threads, side)
        ob = I.make_observation(O.vfield(d, rows[0]), 5.0, I.rng_for(6, side, 1),
                                flux_frac=I.GHASP_FLUX_FRAC, random_mask=I.GHASP_HOLES, W=0.0)
        t0 = time.perf_counter()
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(lambda r: O.vfield_chi2(d, r, ob.vel, ob.sig, ob.evel, ob.esig, ob.mask,
                                                0.0), rows))
        dt = time.perf_counter() - t0
        out["cpu_oracle_512x512"] = {"value": round(len(rows) / dt, 2), "unit": "evals/s",
                                     "cores": threads, "kind": "oracle",
                                     "sample": f"{len(rows)} rows, {dt:.2f} s wall"}
    return out


def line_fit_workload(gbk, I, torch, cpu):
    """Gaussian line fitting of every spectrum (gk_fit_lines): a 128 x 128 x 48
    cube of 16 km/s channels stacked 16 times (262,144 spectra), lines of random
    amplitude, centre and width plus noise; spectra/s and the oracle's rate."""
    nz, dv, crpix, n = 48, 16.0, 24.0, 16 * 128 * 128
    rng = I.rng_for(7, 0, 0)
    amp = torch.tensor(rng.uniform(0.5, 2.0, n), device="cuda")
    mu = torch.tensor(rng.uniform(-200.0, 200.0, n), device="cuda")
    sig = torch.tensor(rng.uniform(15.0, 60.0, n), device="cuda")
    v = (torch.arange(nz, device="cuda", dtype=torch.float64) - crpix) * dv
    noise = torch.tensor(rng.standard_normal((nz, n)), device="cuda")
    cube = (amp * torch.exp(-0.5 * ((v[:, None] - mu) / sig) ** 2) + 0.05 * noise).float().contiguous()
    gbk.fit_lines(cube, 0.0, dv, crpix)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record()
    for _ in range(reps):
        maps, st, it = gbk.fit_lines(cube, 0.0, dv, crpix)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    st, it = st.cpu().numpy(), it.cpu().numpy()
    out = {"workload": "Gaussian line fit of every spectrum: 128x128x48 cube (16 km/s channels) "
                       "x 16, random lines + noise (S/N ~ 10-40)",
           "spectra": n, "ms_per_cube_stack": round(ms, 4), "spectra_per_s": round(n / (ms * 1e-3), 1),
           "mean_trials": round(float(it.mean()), 2),
           "status_fraction": {str(k): round(float((st == k).mean()), 4) for k in range(4)}}
    log(f"line fitting: {n / (ms * 1e-3):.3g} spectra/s")
    if cpu:
        from oracle import fitters as F
        c = cube[:, :200].double().cpu().numpy()
        vv = v.cpu().numpy()
        t0 = time.perf_counter()
        for j in range(c.shape[1]):
            F.fit_gaussian_line(c[:, j], vv, dv)
        dt = time.perf_counter() - t0
        out["cpu_oracle"] = {"value": round(200 / dt, 1), "unit": "spectra/s", "cores": 1,
                             "kind": "oracle", "sample": f"200 spectra, {dt:.2f} s"}
    return out


def large_cube_workload(gbk, I, torch):
    """evals/s on the survey shapes of Sec. 6.5 (SAMI, MaNGA's largest IFU, u = 2)
    and the 700 x 700 high-resolution mock of Sec. 5.3 (u = 1, 15 km/s)."""
    shapes = {
        "sami_32x32x128_u2": (I.Grid(32, 32, 128, 33.5, psf_fwhm=4.2,
                                     lsf_sigma=67.0 / I.FWHM_PER_SIGMA, u=2), 400),
        "manga_64x64x64_u2": (I.Grid(64, 64, 64, 60.0, psf_fwhm=5.0,
                                     lsf_sigma=120.0 / I.FWHM_PER_SIGMA, u=2), 400),
        "hires_700x700x64": (I.Grid(700, 700, 64, 15.0, psf_fwhm=3.0,
                                    lsf_sigma=15.0 / I.FWHM_PER_SIGMA), 200),
    }
    out = {}
    for name, (grid, B) in shapes.items():
        side = min(grid.nx, grid.ny)
        rng = I.rng_for(8, 0, len(out))
        rows = I.c1_box_draw(rng, B, side, grid.psf_fwhm)
        rows[:, I.XO] = rng.uniform(0.45, 0.55, B) * grid.nx
        rows[:, I.YO] = rng.uniform(0.45, 0.55, B) * grid.ny
        rows[:, I.R0] = rng.uniform(0.1, 0.2, B) * side
        rows[:, I.RT] = rng.uniform(0.05, 0.15, B) * side
        m = gbk.Model.from_grid(grid)
        dev = torch.tensor(rows, device="cuda")
        mp = m.evaluate(dev[:1]).cpu().numpy()[0]
        m.set_obs(I.make_observation(mp, 5.0, I.rng_for(8, 1, len(out)), W=0.2))
        c2 = torch.empty(B, dtype=torch.float64, device="cuda")
        nv = torch.empty(B, dtype=torch.int64, device="cuda")
        s = torch.cuda.current_stream()
        for _ in range(2):
            m.chi2(dev, out=c2, n_valid=nv, stream=s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            m.chi2(dev, out=c2, n_valid=nv, stream=s)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 5
        out[name] = {"batch": B, "ms_per_launch": round(1e3 * dt, 3), "evals_per_s": round(B / dt, 1),
                     "conv": m.conv_path()}
        log(f"{name}: {B / dt:.0f} evals/s")
    return out


def log(msg):
    """Progress line on stderr (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def fits_per_hour(gbk, I, torch, n_gal, train_rows):
    """Surrogate workload: training, then plain and screened nested-sampling fits."""
    grid = I.c5_grid()
    m = gbk.Model.from_grid(grid)
    lo, hi = I.c5_box()
    free = list(I.C5_FREE)
    dev = torch.device("cuda:0")
    batch = 512
    steps = max(1, train_rows // batch)
    S = gbk.Surrogate(m, lo, hi, hidden=1024, layers=4, batch=batch, lr=1e-3, lr_final=1e-5, seed=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = S.train(steps)
    t_train = time.perf_counter() - t0
    log(f"surrogate trained on {steps * batch} rows in {t_train:.1f} s")
    out = {"workload": "64x64x64 instrument, 30 km/s channels, PSF FWHM 2.5 px, LSF sigma 30 km/s, "
                       "noise 5 km/s; nested sampling with 1000 live points, 10 free parameters, "
                       f"adaptive batch (1000-16000 candidates, ~{ACCEPT_TARGET} acceptances per round); "
                       f"screen margin 25, audit 2%, rounds screened where it pays (cost {SCREEN_COST}, "
                       f"fixed {SCREEN_ROWS} rows)",
           "train": {"rows": steps * batch, "seconds": round(t_train, 3),
                     "rows_per_s": round(steps * batch / t_train, 1),
                     "final_loss": float(np.mean(losses[-50:]))}}
    fits = []
    # galaxies 0, 1, ... of the workload, none left out; each fit's wall time is
    # capped at FIT_CAP_S (near face-on or dispersion-dominated discs carry the
    # i-Vt degeneracy of Sec. 6.1 and can take the sampler far longer); a capped
    # fit counts with its capped time and is reported as capped
    for k in range(n_gal):
        truth = I.c5_galaxy(k)
        maps = m.evaluate(torch.tensor(truth[None], device=dev)).cpu().numpy()[0]
        obs = I.make_observation(maps, 5.0, I.rng_for(5, k, 1))
        m.set_obs(obs)
        pl = m.fit_nested(lo, hi, free, truth, n_live=1000, batch_max=16000,
                          accept_target=ACCEPT_TARGET, seed=100 + k, max_wall_s=FIT_CAP_S)
        sc = S.fit_nested(m, lo, hi, free, truth, margin=25.0, audit=0.02, n_live=1000,
                          batch_max=16000, accept_target=ACCEPT_TARGET, seed=100 + k,
                          screen_cost=SCREEN_COST, screen_rows=SCREEN_ROWS, max_wall_s=FIT_CAP_S)
        log(f"surrogate workload galaxy {k}: plain {pl['t_wall_s']:.2f} s, screened {sc['t_wall_s']:.2f} s")
        sd = np.where(pl["sd"] > 0, pl["sd"], 1.0)
        fits.append({"galaxy": k, "i_deg": round(float(truth[I.INC]), 1),
                     "vt_sini_over_sigma": round(float(truth[I.VT] * np.sin(np.radians(truth[I.INC]))
                                                       / truth[I.SIG]), 2),
                     "plain_capped": pl["status"] != 0, "screened_capped": sc["status"] != 0,
                     "plain_s": pl["t_wall_s"], "screened_s": sc["t_wall_s"],
                     "plain_rounds": pl["n_launches"], "screened_rounds": sc["n_launches"],
                     "plain_wait_s": pl["t_wait_s"], "screened_wait_s": sc["t_wait_s"],
                     "plain_evals": pl["n_evals"], "screened_plain_evals": sc["n_evals"],
                     "surrogate_evals": sc["n_screened"], "audit_misses": sc["n_audit_miss"],
                     "max_median_shift_sd": float(np.max(np.abs(sc["median"] - pl["median"]) / sd))})
    if fits:
        tp = sum(f["plain_s"] for f in fits)
        ts = sum(f["screened_s"] for f in fits)
        out.update({"galaxies": len(fits), "selection": "first galaxies of the workload, unfiltered",
                    "cap_s_per_fit": FIT_CAP_S,
                    "plain_capped": sum(f["plain_capped"] for f in fits),
                    "screened_capped": sum(f["screened_capped"] for f in fits),
                    "plain": round(3600 * len(fits) / tp, 1),
                    "screened": round(3600 * len(fits) / ts, 1), "ratio": round(tp / ts, 3),
                    "unit": "fits/hour", "fits": fits})
    S.close()
    return out


def surrogate_kernels(gbk, I, torch, reps=10):
    """The surrogate's kernels at the screening shape: the BF16 GEMM on an
    8192 x 8192 x 1024 product (the output layer's shape with every pixel
    kept) and the screening pass, i.e. the surrogate chi-square of 8192 rows of
    the 64x64x64 instrument (encoding, 4 x 1024 GELU layers, output layer with
    the fused chi-square), against the dense BF16 MFMA peak."""
    dev = "cuda:0"
    g = torch.Generator(device=dev).manual_seed(1)
    A = torch.randn(8192, 1024, device=dev, generator=g).to(torch.bfloat16)
    Bm = torch.randn(8192, 1024, device=dev, generator=g).to(torch.bfloat16)
    C = torch.empty(8192, 8192, device=dev, dtype=torch.float32)

    def timed(fn):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    t_gemm = timed(lambda: gbk.gemm_bf16(A, Bm, C=C))
    gemm_tflops = 2 * 8192 * 8192 * 1024 / t_gemm / 1e12
    del A, Bm, C
    grid = I.c5_grid()
    m = gbk.Model.from_grid(grid)
    lo, hi = I.c5_box()
    truth = I.c5_galaxy(1)
    maps = m.evaluate(torch.tensor(truth[None], device=dev)).cpu().numpy()[0]
    m.set_obs(I.make_observation(maps, 5.0, I.rng_for(5, 1, 1)))
    S = gbk.Surrogate(m, lo, hi, hidden=1024, layers=4, batch=512, seed=1)
    rows = torch.tensor(lo + I.rng_for(5, 0, 9).random((8192, I.NPAR)) * (hi - lo), device=dev)
    t_scr = timed(lambda: S.chi2(m, rows))
    t_plain = timed(lambda: m.chi2(rows))
    S.close()
    m.close()
    return {"gemm_8192x8192x1024": {"us": round(t_gemm * 1e6, 1), "tflops": round(gemm_tflops, 1),
                                   "frac_of_bf16_peak": round(gemm_tflops / PEAK_BF16_TFLOPS, 4)},
            "screen_8192_rows": {"us": round(t_scr * 1e6, 1), "ns_per_row": round(t_scr / 8192 * 1e9, 2)},
            "plain_8192_rows": {"us": round(t_plain * 1e6, 1), "ns_per_row": round(t_plain / 8192 * 1e9, 2)},
            "peak_bf16_tflops": PEAK_BF16_TFLOPS}


def host_threads() -> int:
    """Host threads for the oracle legs: the CPUs this process may run on,
    at most 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def host_info() -> dict:
    """CPU model, clock and counts of the host that runs the oracle."""
    info = {"nproc": os.cpu_count(), "usable_cpus": host_threads()}
    try:
        with open("/proc/cpuinfo") as f:
            txt = f.read()
        for line in txt.splitlines():
            if line.startswith("model name") and "cpu_model" not in info:
                info["cpu_model"] = line.split(":", 1)[1].strip()
            if line.startswith("cpu MHz") and "cpu_mhz_now" not in info:
                info["cpu_mhz_now"] = float(line.split(":", 1)[1])
    except OSError:
        pass
    try:
        with open("/sys/devices/system/cpu/cpu0/cpufreq/cpuinfo_max_freq") as f:
            info["cpu_mhz_max"] = int(f.read()) / 1000.0
    except (OSError, ValueError):
        pass
    return info


def cpu_baseline(grid, first_row, obs, st_rows, mt_rows_per_thread, reps=3):
    """The FP64 oracle (untuned) on bounded samples of the same workload, like
    the paper's ST and MT setups (Sec. 5.1): one core, then every usable core
    with one evaluation per thread; the median of `reps` runs each.  The
    samples are `first_row` (also evaluated on the GPU, for a cross-check)
    plus rows drawn like the timed batches."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import oracle as O
    from paper_1510_01815_amd import inputs as I
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from parity import oracle_desc
    O.lib()
    d = oracle_desc(O, grid.as_dict())
    threads = host_threads()
    n_mt = threads * mt_rows_per_thread
    sample = np.concatenate([first_row[None, :],
                             I.c2_draw(I.rng_for(2, 0, 3), max(n_mt, st_rows) - 1)])

    def one(r):
        return O.eval_chi2(d, r, obs.vel, obs.sig, obs.evel, obs.esig, obs.mask, obs.W)[0]

    st, mt, res = [], [], None
    for _ in range(reps):
        t0 = time.perf_counter()
        res = [one(r) for r in sample[:st_rows]]
        st.append(st_rows / (time.perf_counter() - t0))
    for _ in range(reps):
        t0 = time.perf_counter()
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(one, sample[:n_mt]))
        mt.append(n_mt / (time.perf_counter() - t0))
    v_mt, v_st = float(np.median(mt)), float(np.median(st))
    return {"value": round(v_mt, 2), "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_mt} rows drawn like the timed batches ({mt_rows_per_thread} per thread, "
                      f"one evaluation per thread), FP64 literal cube pipeline; median of {reps} "
                      f"runs ({', '.join(f'{v:.1f}' for v in mt)} evals/s)",
            "single_core": {"value": round(v_st, 2), "unit": "evals/s", "cores": 1,
                            "sample": f"{st_rows} rows on one thread, median of {reps} runs "
                                      f"({', '.join(f'{v:.2f}' for v in st)} evals/s)"},
            "host": host_info(), "chi2_first": res[0]}


def precision_study(samples):
    """Per-map largest deviation of the GPU's maps from the FP64 oracle's on
    sampled nodes of the beam-smeared grid workload: m0 relative, m1 and m2
    in km/s, over spaxels whose oracle flux is at least 1e-12 of the map's
    peak (fainter ones must only be finite)."""
    from oracle import oracle as O
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from parity import oracle_desc
    O.lib()
    worst = {"m0_rel": 0.0, "m1_kms": 0.0, "m2_kms": 0.0}
    n = 0
    for grid, rows, gpu in samples:
        d = oracle_desc(O, grid.as_dict())
        for r, g in zip(rows, gpu):
            ref = O.evaluate(d, r)
            b = ref[0] >= 1e-12 * np.nanmax(ref[0])
            g = g.astype(np.float64)
            assert np.isfinite(g).all()
            worst["m0_rel"] = max(worst["m0_rel"], float(np.max(np.abs(g[0] - ref[0])[b] / ref[0][b])))
            worst["m1_kms"] = max(worst["m1_kms"], float(np.max(np.abs(g[1] - ref[1])[b])))
            worst["m2_kms"] = max(worst["m2_kms"], float(np.max(np.abs(g[2] - ref[2])[b])))
            n += 1
    return {"nodes": n, "galaxies": len(samples), **{k: float(f"{v:.3g}") for k, v in worst.items()},
            "bar": {"m0_rel": 1e-5, "m1_kms": "1e-3 + 1e-5 |m1|", "m2_kms": "1e-3 + 1e-5 |m2|"},
            "precision": "FP32 exp2 / rotation curve, FP64 radius, sums, PSF passes, moments"}


def oracle_rate_c5(I):
    """The oracle's evals/s on the surrogate workload's instrument (2 rows per thread)."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import oracle as O
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from parity import oracle_desc
    O.lib()
    grid = I.c5_grid()
    d = oracle_desc(O, grid.as_dict())
    lo, hi = I.c5_box()
    truth = I.c5_galaxy(1)
    obs = I.make_observation(O.evaluate(d, truth), 5.0, I.rng_for(5, 1, 1))
    threads = host_threads()
    rows = lo + I.rng_for(5, 0, 9).random((threads * 2, I.NPAR)) * (hi - lo)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(lambda r: O.eval_chi2(d, r, obs.vel, obs.sig, obs.evel, obs.esig, obs.mask,
                                          obs.W), rows))
    return len(rows) / (time.perf_counter() - t0), threads


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); "
              "this build has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1510_01815_amd import gbk
    from paper_1510_01815_amd import inputs as I
    if not os.path.exists(gbk.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    dev = torch.device("cuda:0")

    grid = I.c2_grid()
    model = gbk.Model.from_grid(grid, device=0)
    truth = I.c2_draw(I.rng_for(2, 0, 0), 1)
    truth_maps = model.evaluate(torch.tensor(truth, device=dev)).cpu().numpy()[0]
    obs = I.make_observation(truth_maps, 3.0, I.rng_for(2, 0, 1))
    model.set_obs(obs)

    tune = model.autotune(BATCH)  # launch shape of the PSF/moment stage, timed on this GPU
    log(f"autotuned: {tune['conv']} {tune['tile']}")
    K, W = args.steps, args.warmup
    rng = I.rng_for(2, 0, 2)
    batches = torch.tensor(I.c2_draw(rng, (K + W) * BATCH).reshape(K + W, BATCH, I.NPAR),
                           device=dev)
    chi2 = torch.empty((K + W, BATCH), dtype=torch.float64, device=dev)
    nval = torch.empty((K + W, BATCH), dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()

    for k in range(W):
        model.chi2(batches[k], out=chi2[k], n_valid=nval[k], stream=stream)
    torch.cuda.synchronize()

    # timed region: K steps; the launches of every TIME_EVERY-th step carry HIP
    # events on `stream` (an event-carrying dispatch leaves the GPU idle for
    # ~9 us before the next one, so timing every step would slow the job)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, k in enumerate(range(W, W + K)):
        model.set_profiling(gbk.GK_PROF_TIMING if i % TIME_EVERY == 0 else 0)
        model.chi2(batches[k], out=chi2[k], n_valid=nval[k], stream=stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    model.set_profiling(0)
    prof = model.read_profile()

    # untimed pass over the same batches: count the line-support voxels
    model.set_profiling(gbk.GK_PROF_COUNT)
    for k in range(W, W + K):
        model.chi2(batches[k], stream=stream)
    torch.cuda.synchronize()
    cnt = model.read_profile()
    model.set_profiling(0)

    assert torch.isfinite(chi2[W:]).all().item(), "non-finite chi-square in the timed steps"
    evals = K * BATCH
    value = evals / dt

    per_kernel_ms = {n: prof["kernel_ms"][n] / max(prof["launches"][n], 1)
                     for n in gbk.KERNEL_NAMES}
    nxe, nye, _, _, _ = model.dims()
    # k_line_sums: the algorithmic model above, per launch: every fine spaxel of
    # every row, and the line-support voxels counted in the untimed pass
    ls_ms = per_kernel_ms["k_line_sums"]
    vox_per_launch = cnt["support_voxels"] / K
    spx_per_launch = BATCH * nxe * nye
    ls_flop = spx_per_launch * SPAXEL_FLOP + vox_per_launch * FLOP_PER_VOXEL
    ls_tflops = ls_flop / (ls_ms * 1e-3) / 1e12
    ls_slots = spx_per_launch * SPAXEL_SLOTS + vox_per_launch * VOXEL_SLOTS
    ls_slot_frac = ls_slots / (ls_ms * 1e-3) / LANE_OPS_PER_S
    counters = measured_counters()
    # k_psf_moments: algorithmic HBM bytes = the three T planes of every row
    # read once, plus the observation and the tile partials
    ps_ms = per_kernel_ms["k_psf_moments"]
    ps_bytes = BATCH * 3 * nxe * nye * 8 + 128 * 128 * 25 + BATCH * 32 * 8
    ps_gbs = ps_bytes / (ps_ms * 1e-3) / 1e9
    def valu_issue(name, ms):
        c = counters.get(name)
        if not c or not c.get("SQ_INSTS_VALU"):
            return None
        return round(c["SQ_INSTS_VALU"] / (ms * 1e-3) / VALU_ISSUE_PER_S, 4)

    rooflines = {
        "k_line_sums": {"bound": "alu", "kernel": "k_line_sums", "achieved": round(ls_tflops, 3),
                        "peak": round(PEAK_TFLOPS, 1), "unit": "TFLOP/s",
                        "frac": round(ls_tflops / PEAK_TFLOPS, 4),
                        "traffic": counters.get("k_line_sums", {}).get("hbm_bytes"),
                        "kernel_ms_avg": round(ls_ms, 5),
                        "model": f"{SPAXEL_FLOP} FP64 FLOP ({SPAXEL_SLOTS} VALU slots) per fine "
                                 f"spaxel + {FLOP_PER_VOXEL} FP64 FLOP ({VOXEL_SLOTS} slots) per "
                                 "line-support voxel",
                        "spaxels_per_launch": spx_per_launch,
                        "support_voxels_per_launch": int(vox_per_launch),
                        "issue_slot_frac": round(ls_slot_frac, 4),
                        "valu_issue_frac_measured": valu_issue("k_line_sums", ls_ms)},
        "k_psf_moments": {"bound": "hbm", "kernel": "k_psf_moments", "achieved": round(ps_gbs, 1),
                          "peak": PEAK_HBM_GBS, "unit": "GB/s",
                          "frac": round(ps_gbs / PEAK_HBM_GBS, 4),
                          "traffic": counters.get("k_psf_moments", {}).get("hbm_bytes"),
                          "kernel_ms_avg": round(ps_ms, 5),
                          "algorithmic_bytes_per_launch": ps_bytes,
                          "valu_issue_frac_measured": valu_issue("k_psf_moments", ps_ms)},
    }
    dominant = max(("k_line_sums", "k_psf_moments"), key=lambda n: per_kernel_ms[n])
    roofline = rooflines[dominant]
    per_kernel_ms = {n: round(v, 5) for n, v in per_kernel_ms.items()}

    out = {"metric": METRIC, "value": round(value, 1), "unit": "evals/s", "n_gpus": 1,
           "steps": K, "warmup": W, "ms_per_step": round(1e3 * dt / K, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32 exp / f64 sums", "data": "synthetic",
           "config": {"workload": "Fabry-Perot-like 128x128x48 cube, 16 km/s channels, "
                                  "400 nested-sampling proposals per launch",
                      "nx": 128, "ny": 128, "nz": 48, "batch": BATCH,
                      "psf_fwhm_pix": grid.psf_fwhm, "lsf_sigma_kms": round(grid.lsf_sigma, 4),
                      "rotation_curve": "exponential rise", "parallelism": "single GPU",
                      "conv": tune["conv"], "tile": list(tune["tile"])},
           "roofline": roofline, "rooflines": rooflines, "kernel_ms_per_launch": per_kernel_ms,
           "kernel_timing": f"HIP events carried by the dispatches of every {TIME_EVERY}th "
                            f"timed step ({prof['launches']['k_line_sums']} launches per kernel)"}
    log(f"{value:.0f} evals/s on the 128x128x48 workload")
    if args.fit_galaxies > 0 or args.surrogate_kernels_only:
        out["surrogate_kernels"] = surrogate_kernels(gbk, I, torch)
        log(f"surrogate kernels: {out['surrogate_kernels']}")
    if args.fit_galaxies > 0 and not args.surrogate_kernels_only:
        out["fits_per_hour"] = fits_per_hour(gbk, I, torch, args.fit_galaxies, args.train_rows)
    precision_samples = []
    if args.survey_galaxies > 0 or args.grid_galaxies > 0 or args.ns_fits > 0:
        out["workloads"] = other_workloads(gbk, I, torch, args.survey_galaxies, args.grid_galaxies,
                                           args.ns_fits, precision_samples)
    if not args.no_large_cubes:
        out["large_cubes"] = large_cube_workload(gbk, I, torch)
    if not args.no_line_fit:
        out["line_fitting"] = line_fit_workload(gbk, I, torch, not args.no_cpu_baseline)
    if args.vfield_galaxies >= 0:
        out["velocity_field"] = velocity_field_workload(gbk, I, torch, args.vfield_galaxies,
                                                        not args.no_cpu_baseline)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(grid, batches[W, 0].cpu().numpy(), obs,
                                           args.cpu_rows_single, args.cpu_rows_per_thread)
        log(f"oracle: {out['cpu_baseline']['value']:.1f} evals/s on {out['cpu_baseline']['cores']} "
            f"cores, {out['cpu_baseline']['single_core']['value']:.2f} on one")
        if precision_samples:
            out["precision_30x30x64"] = precision_study(precision_samples)
        gpu_first = float(chi2[W, 0].item())
        cb = out["cpu_baseline"].pop("chi2_first")
        out["cpu_baseline"]["chi2_rel_diff_first_row"] = abs(gpu_first - cb) / abs(cb)
        fph = out.get("fits_per_hour", {})
        if fph.get("fits"):
            evals = float(np.mean([f["plain_evals"] for f in fph["fits"]]))
            eps, threads = oracle_rate_c5(I)
            out["cpu_baseline"]["surrogate_workload"] = {
                "evals_per_s": round(eps, 2), "cores": threads,
                "fits_per_hour": round(3600 * eps / evals, 4),
                "kind": "extrapolated: oracle evals/s on the 64x64x64 instrument x the plain "
                        "fitter's evaluations per fit"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
