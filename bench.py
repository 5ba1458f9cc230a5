"""Benchmark of the GRHD Runge-Kutta substep on one MI355X.

Headline workload: the perturbed TOV star (K = 100, Gamma = 2,
rho_c = 1.28e-3, Cowling metric) on a 1024 x 1024 cylindrical grid covering
[0, 20]^2, PPM + HLLC, SSP-RK3, the paper's face states.  A benchmark step
is one full SSP-RK3 time step = three substeps, with the diagnostics on.
Inputs are resident in HBM before the timed region.

Metric: zone-updates/s (interior cells x substeps / second) of the plain
FP64 path, in the faster of its two forms (config.form):
  forms.fp64     each substep a recovery pass, the fused reconstruction /
                 flux / divergence / source / stage kernel and the
                 diagnostic fold (grhd_rk_substep);
  forms.fp64_chained  each substep one chained kernel (grhd_rk_substep_chained:
                 the stage, then the recovery of the new state) and the fold;
                 one recovery pass starts the chain.
The JSON line also carries:
  forms.mixed    FP32 reconstruction and flux, FP64 recovery and update, in
                 the chained form, with its L1 error against the FP64 path
                 after N substeps;
  forms.combined the headline star through the form the three patterns
                 combine into: mixed precision, the batched plan (one
                 graph-captured launch sequence per substep) and the learned
                 recovery guess (the matrix-core MLP trained here on GPU on
                 star-like states), with and without the guess, and the
                 chained mixed stage with and without the guess, against the
                 plain FP64 headline: zone-updates/s, speedup, and the L1
                 difference from the FP64 path after N substeps;
  forms.batched  six nested 256^2 star levels plus 64 Riemann patches
                 (N_x log-uniform in [128, 2048], 8 periodic z cells) in one
                 graph-captured batched launch, against one call per patch;
  forms.fmr      Berger-Oliger evolution of the same six levels as one
                 refinement hierarchy (prolongation at every stage,
                 restriction, refluxing; l_fix = 0 and l_fix = 5), with the
                 composite baryon-mass change over the timed steps;
  forms.bondi    Bondi accretion in the maximal trumpet slice (shift, lapse
                 and extrinsic curvature all active) on [0, 16M]^2 to t = 20M
                 at N = 64, 128, 256: PPM (CW84) and minmod with HLLC, the
                 per-cell third-order parabola (PPM3) with HLLC and TVDLF,
                 PPM and PPM3 with the face eps from the EOS; zone-updates/s
                 and the L1 density error of each, with the convergence
                 orders;
  forms.bondi_rt the hot bubble in the Bondi flow (N = 512, t = 25M), HLLC
                 against TVDLF: total variation of the density (sharper
                 fingers give more) and zone-updates/s;
  forms.general  the general-metric stage at 1024^2: Bondi on the trumpet
                 slice (8 metric arrays) and a 17-array metric; throughput,
                 stage-kernel time and its roofline against the bytes of the
                 metric arrays actually read;
  forms.learned  recovery of a 2048^2 differentially rotating field, Illinois
                 from the bracket against Newton seeded by the matrix-core MLP
                 (trained here on GPU), same root;
  roofline       of the headline's stage kernel (HIP events recorded by the
                 library around that kernel): the algorithmic bytes of one
                 fused pass (96, 136, 136 B per zone over the stages) per
                 mean launch time, with the whole substep's fraction beside it;
  cpu_baseline   the oracle on the host cores (one band of rows per core)
                 and on one core, bounded samples of the headline workload.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--forms fp64,mixed,...]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# bytes per zone that the separate-recovery stage kernel (k_substep) reads
# and writes by design, FP64 fields once: primitives (6 x 8), lapse and W
# (2 x 8), q_s (5 x 8) read, q_out (5 x 8) written; stages 2 and 3 also read
# q^n (5 x 8)
BYTES_KERNEL = [144.0, 184.0, 184.0]
# the same for the chained stage kernel (k_substep_chain): primitives and
# flags of q_s read (49), lapse and W (16), q_s (40) [+ q^n 40]; q_out (40),
# its primitives and flags (49) written
BYTES_CHAINED = [194.0, 234.0, 234.0]
# algorithmic bytes per zone-update of a whole substep (recovery included):
# q_s and the metric read, q_out written, q^n read in stages 2 and 3
BYTES_SUBSTEP = [96.0, 136.0, 136.0]
ALL_FORMS = ("fp64", "fp64_chained", "mixed", "combined", "batched", "fmr", "bondi", "bondi_rt", "general",
             "learned")
# measured HBM traffic of the fused kernel (rocprofv3 FETCH_SIZE/WRITE_SIZE,
# calibrated with a plain copy) is kept with the hash of the sources it was
# measured on; it is reported only while the sources still hash the same
TRAFFIC_FILES = {False: os.path.join(ROOT, "profiles", "k_substep_star1024_counters.md"),
                 True: os.path.join(ROOT, "profiles", "k_substep_chain_star1024_counters.md")}
KERNEL_SOURCES = ["paper_2502_03223_amd/csrc/" + f for f in
                  ("grhd_tile.hpp", "grhd_dev.hpp", "grhd_diag.hpp", "grhd_host.hpp", "grhd_kernels.hip")] + \
                 ["paper_2502_03223_amd/build.py"]


def kernel_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(nzone, chained):
    """(bytes per launch of that stage kernel, bytes per substep of every
    kernel) recorded with its counter profile, or (None, None) when absent,
    taken on other sources or on a launch of another size."""
    try:
        kv = {}
        keys = ("traffic_bytes_per_launch", "traffic_bytes_per_substep", "source_sha256", "zones_per_launch")
        for line in open(TRAFFIC_FILES[chained]):
            if ":" in line and line.split(":", 1)[0].strip() in keys:
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip().strip("`")
        if kv.get("source_sha256") != kernel_sources_hash() or int(kv["zones_per_launch"]) != nzone:
            return None, None
        return float(kv["traffic_bytes_per_launch"]), float(kv["traffic_bytes_per_substep"])
    except (OSError, KeyError, ValueError):
        return None, None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--forms", default=",".join(ALL_FORMS))
    ap.add_argument("--accuracy-substeps", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-reuse-atm", action="store_true",
                    help="the star forms' recoveries rewrite the primitives of every cell")
    ap.add_argument("--cpu-sample-rows", type=int, default=128,
                    help="rows of the single-core oracle sample")
    ap.add_argument("--cpu-sample-steps", type=int, default=3)
    ap.add_argument("--learned-n", type=int, default=2048)
    ap.add_argument("--train-pairs", type=int, default=1 << 20)
    ap.add_argument("--train-steps", type=int, default=10000)
    ap.add_argument("--tile", default="", help="tile shape of the single-patch forms, e.g. 16x8 "
                    "(default: the library's)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run a plain device-to-device copy of this many MiB three "
                         "times (calibrates HBM byte counters against a known size)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    forms = [f for f in args.forms.split(",") if f]
    for f in forms:
        if f not in ALL_FORMS:
            sys.exit("unknown form %r" % f)
    import torch

    import synth
    from paper_2502_03223_amd import grhd

    dev = torch.device("cuda:0")
    if args.copy_mib:
        src = torch.ones(args.copy_mib << 17, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print("copy calibration: %d MiB read + %d MiB written per copy, 3 copies"
              % (args.copy_mib, args.copy_mib), file=sys.stderr)
        del src, dst

    n = args.n
    grid = synth.star_grid(n, extent=20.0)
    tov = synth.tov_solve()
    p_np, metric_np, eos = synth.star_problem(grid, seed=2025, tov=tov)
    metric = {k: torch.from_numpy(v).to(dev) for k, v in metric_np.items()}
    # cells that stay atmosphere keep the primitives of the previous
    # recovery into the same buffer (bit for bit the same p)
    c2p = dict(w_max=100.0, rho_atm=1e-10, reuse_atm=not args.no_reuse_atm)
    dt = 0.4 * grid["dx"]
    nzone = grid["nx"] * grid["nz"]

    def make_state():
        p = torch.from_numpy(p_np).to(dev)
        q = torch.zeros((5,) + p.shape[1:], dtype=torch.float64, device=dev)
        grhd.prim2con(grid, eos, metric, p, q, with_ghosts=True)
        return q

    class Stepper:
        """SSP-RK3 steps of the star, chained (one kernel per substep, the
        recovery at the end of each stage) or separate (recovery pass, then
        the stage kernel)."""

        def __init__(self, prec, chained=True, mlp=None):
            cp = dict(c2p, mlp=mlp)
            opts = dict(recon="ppm", riemann="hllc", prec=prec, c2p=cp)
            if args.tile and not chained:
                opts["tile"] = tuple(int(v) for v in args.tile.split("x"))
            self.chained = chained
            self.sub = grhd.Substep(grid, eos, metric, opts)
            self.q = make_state()
            self.q1 = torch.zeros_like(self.q)
            self.q2 = torch.zeros_like(self.q)
            shp = self.q.shape[1:]
            self.p = torch.zeros((6,) + shp, dtype=torch.float64, device=dev)
            self.pb = torch.zeros_like(self.p)
            self.fa = torch.zeros(shp, dtype=torch.uint8, device=dev)
            self.fb = torch.zeros_like(self.fa)
            self.diag = grhd.new_diag()
            self.stages = [grhd.make_stage(dict(s, dt=dt)) for s in grhd.SSPRK3]
            if chained:
                grhd.con2prim(grid, eos, metric, cp, self.q, self.p, flags=self.fa)

        def step(self, events=None, kevents=None):
            # q -> q1 -> q2 -> q (SSP-RK3, q^n = q)
            bufs = [(self.q, self.q, self.q1), (self.q, self.q1, self.q2), (self.q, self.q2, self.q1)]
            prims = [(self.p, self.fa, self.pb, self.fb), (self.pb, self.fb, self.p, self.fa),
                     (self.p, self.fa, self.pb, self.fb)]
            for s, (qn, qs, qo) in enumerate(bufs):
                if events is not None:
                    events[s][0].record()
                kev = kevents[s] if kevents is not None else None
                if self.chained:
                    self.sub.chained(self.stages[s], qn, qs, qo, *prims[s], diag=self.diag, events=kev)
                else:
                    self.sub(self.stages[s], qn, qs, qo, self.p, flags=self.fa, diag=self.diag, events=kev)
                if events is not None:
                    events[s][1].record()
            self.q, self.q1 = self.q1, self.q
            if self.chained:
                self.p, self.pb = self.pb, self.p
                self.fa, self.fb = self.fb, self.fa

        def prims(self):
            """Primitives of the current state."""
            if not self.chained:
                grhd.con2prim(grid, eos, metric, c2p, self.q.clone(), self.p)
            return self.p

    def run_form(prec, chained=True):
        st = Stepper(prec, chained)
        for _ in range(args.warmup):
            st.step()
        torch.cuda.synchronize()
        # 1. throughput: K steps with nothing recorded on the stream (every
        #    event record adds a gap of several microseconds between kernels)
        t0 = time.perf_counter()
        for k in range(args.steps):
            st.step()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        # 2. the same K steps again with events: torch events around each
        #    substep (stage time) and HIP events the library records around
        #    the fused kernel (kernel time, for the roofline)
        evs = [[[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(3)]
               for _ in range(args.steps)]
        kevs = [[(grhd.Event(), grhd.Event()) for _ in range(3)] for _ in range(args.steps)]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for k in range(args.steps):
            st.step(evs[k], kevs[k])
        torch.cuda.synchronize()
        wall_ev = time.perf_counter() - t1
        stage_ms = np.array([[evs[k][s][0].elapsed_time(evs[k][s][1]) for s in range(3)]
                             for k in range(args.steps)])
        kernel_ms = np.array([[kevs[k][s][0].elapsed_ms(kevs[k][s][1]) for s in range(3)]
                              for k in range(args.steps)])
        return dict(wall=wall, wall_with_events=wall_ev, stage_ms=stage_ms.mean(axis=0),
                    kernel_ms=kernel_ms.mean(axis=0), diag=grhd.read_diag(st.diag))

    out_forms = {}
    # the plain FP64 path in its two forms: separate recovery pass + stage
    # kernel, and the chained stage (recovery of the new state at the end of
    # each stage kernel); the headline is the faster of the two
    res64 = {}
    for chained in (False, True):
        r = run_form("fp64", chained=chained)
        res64[chained] = r
        key = "fp64_chained" if chained else "fp64"
        v = 3 * nzone * args.steps / r["wall"]
        out_forms[key] = {"value": v, "ms_per_step": r["wall"] * 1e3 / args.steps, "chained": chained,
                          "ms_per_step_with_events": r["wall_with_events"] * 1e3 / args.steps,
                          "kernel_ms": r["kernel_ms"].tolist(), "stage_ms": r["stage_ms"].tolist()}
        print("%s done: %.3e zone-updates/s" % (key, v), file=sys.stderr, flush=True)
    head_chained = res64[True]["wall"] < res64[False]["wall"]
    r64 = res64[head_chained]
    value = 3 * nzone * args.steps / r64["wall"]
    ms_per_step = r64["wall"] * 1e3 / args.steps
    # roofline of the headline's stage kernel: the algorithmic bytes of one
    # fused pass over a zone (q_s and lapse, W read, q_out written, q^n read
    # in stages 2 and 3: 96, 136, 136 B) over that kernel's mean duration
    kms = float(r64["kernel_ms"].mean())
    bytes_per_launch = float(np.mean(BYTES_SUBSTEP)) * nzone
    achieved = bytes_per_launch / (kms * 1e-3) / 1e9
    # the same bytes over the whole substep's wall time (every kernel of it,
    # fold included, from the clean pass)
    substep_gbs = float(np.mean(BYTES_SUBSTEP)) * nzone / (ms_per_step / 3.0 * 1e-3) / 1e9
    diag = r64["diag"]
    tb, tsub = measured_traffic(nzone, head_chained)
    traffic = tb / (kms * 1e-3) / 1e9 if tb else None
    # every kernel of a substep (recovery, stage, fold) over its wall time
    traffic_substep = tsub / (ms_per_step / 3.0 * 1e-3) / 1e9 if tsub else None
    if "mixed" in forms:
        rm = run_form("mixed")
        value_m = 3 * nzone * args.steps / rm["wall"]
        out_forms["mixed"] = {"value": value_m, "ms_per_step": rm["wall"] * 1e3 / args.steps, "chained": True,
                              "speedup_vs_fp64": value_m / value,
                              "kernel_ms": rm["kernel_ms"].tolist(),
                              "accuracy_vs_fp64": mixed_accuracy(args, Stepper, grid, eos, metric,
                                                                 metric_np, c2p)}
        print("mixed done", file=sys.stderr, flush=True)
    if "combined" in forms:
        out_forms["combined"] = combined_form(args, grid, eos, metric, metric_np, make_state, value, Stepper)
        print("combined done", file=sys.stderr, flush=True)
    if "batched" in forms:
        out_forms["batched"] = batched_form(args, tov)
        print("batched done", file=sys.stderr, flush=True)
    if "fmr" in forms:
        out_forms["fmr"] = fmr_form(args, tov)
        print("fmr done", file=sys.stderr, flush=True)
    if "bondi" in forms:
        out_forms["bondi"] = bondi_form(args)
        print("bondi done", file=sys.stderr, flush=True)
    if "bondi_rt" in forms:
        out_forms["bondi_rt"] = bondi_rt_form(args)
        print("bondi_rt done", file=sys.stderr, flush=True)
    if "general" in forms:
        out_forms["general"] = general_form(args)
        print("general done", file=sys.stderr, flush=True)
    if "learned" in forms:
        out_forms["learned"] = learned_form(args)
        print("learned done", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(grid, eos, metric_np, p_np, c2p, dt, args.cpu_sample_steps, args.cpu_sample_rows)

    out = {
        "metric": "zone-updates/s per GRHD RK substep at 1 GPU, FP64 plain vs mixed/batched",
        "value": value,
        "unit": "zone-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "TOV star K=100 Gamma=2 rho_c=1.28e-3, %dx%d cylindrical [0,20]^2, "
                        "Cowling metric, PPM+HLLC, SSP-RK3 (3 substeps per step)" % (n, n),
            "zones": nzone, "substeps_per_step": 3, "seed": 2025,
            "form": "chained" if head_chained else "separate recovery",
            "face_states": "reconstructed rho, u_i, P, eps",
            "recovery_reuse_atm": not args.no_reuse_atm,
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": ("k_substep_chain<double> (reconstruction, flux, divergence, sources, stage, "
                       "then the recovery of the new state)" if head_chained else
                       "k_substep<double> (reconstruction, flux, divergence, sources, stage)"),
            "form": "chained" if head_chained else "separate recovery",
            "bytes_per_zone": BYTES_SUBSTEP, "kernel_ms": r64["kernel_ms"].tolist(),
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "kernel_design_bytes_per_zone": BYTES_CHAINED if head_chained else BYTES_KERNEL,
            "kernel_design_gbs": float(np.mean(BYTES_CHAINED if head_chained else BYTES_KERNEL)) * nzone
                                 / (kms * 1e-3) / 1e9,
            "measured_bytes_per_launch": tb,
            "measured_bytes_per_substep": tsub, "traffic_substep": traffic_substep,
            "substep_gbs": substep_gbs, "substep_frac": substep_gbs / HBM_PEAK_GBS,
            "bytes_note": "achieved = the algorithmic bytes of one fused pass (96, 136, 136 B per zone "
                          "over the three SSP-RK3 stages) x zones / mean kernel time; "
                          "kernel_design_gbs counts what this kernel reads and writes by design "
                          "(primitives and flags of the chained form, or the primitive re-read of "
                          "the separate-recovery form) over the same time",
            "traffic_note": "traffic = measured HBM bytes per launch (FETCH x2 + WRITE x1, factors "
                            "from a 256 MiB copy) / the same mean launch time, in GB/s; traffic_substep = "
                            "the measured bytes of every kernel of a substep (recovery, stage, fold) / the "
                            "substep's wall time; null when the kernel sources changed since the counters "
                            "were taken",
            "timing_note": "value and ms_per_step come from K steps with nothing recorded on the stream; "
                           "kernel_ms and stage_ms from the same K steps repeated right after with HIP "
                           "events around every fused kernel and every substep",
        },
        "forms": out_forms,
        "diag_last_stage": dict({k: diag[k] for k in ("max_courant", "Mb", "n_atm", "n_cold",
                                                       "n_rescale", "iter_max")},
                                iter_mean=diag["iter_sum"] / nzone),
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def mixed_accuracy(args, Stepper, grid, eos, metric, metric_np, c2p):
    """L1 differences of the mixed form from the FP64 path after the same
    number of substeps from the same initial data."""
    import synth
    nsteps = args.accuracy_substeps // 3
    a64, a32 = Stepper("fp64", chained=False), Stepper("mixed")
    for _ in range(nsteps):
        a64.step()
        a32.step()
    P64 = synth.interior(grid, a64.prims().cpu().numpy())
    P32 = synth.interior(grid, a32.prims().cpu().numpy())
    X, _ = synth.cell_coords(grid)
    x = synth.interior(grid, X)
    Wm = synth.interior(grid, metric_np["W"])
    alp = synth.interior(grid, metric_np["alp"])
    wgt = alp * Wm ** -3 * x           # sqrt(-g) dV / (2 pi dx dz)

    def l1rel(a, b):
        return float((np.abs(a - b) * wgt).sum() / (np.abs(b) * wgt).sum())

    def vel(P):
        w = np.sqrt(1.0 + Wm ** 2 * (P[1] ** 2 + P[2] ** 2 + P[3] ** 2))
        return Wm ** 2 * P[1] / w, Wm ** 2 * P[3] / w
    vx64, vz64 = vel(P64)
    vx32, vz32 = vel(P32)
    l1_v = float(((np.abs(vx32 - vx64) + np.abs(vz32 - vz64)) * x).sum() / x.sum())
    return dict(substeps=3 * nsteps, l1_rel_rho=l1rel(P32[0], P64[0]),
                l1_rel_eps=l1rel(P32[5], P64[5]), l1_abs_v=l1_v,
                max_abs_v_fp64=float(np.abs(np.stack([vx64, vz64])).max()))


def train_guess(samples, eos, seed, train_steps, dev):
    """The learned recovery guess trained on GPU with the library's kernels:
    (D, S, tau) -> P pairs through the library's prim->con of the sampled
    states.  Returns (network, training record)."""
    import torch

    import synth
    from paper_2502_03223_amd import grhd
    npair = samples.shape[0]
    tg = synth.make_grid(npair, 1, 0.0, 0.0, 1.0, 1.0, "cart", ("outflow",) * 4)
    ng = tg["ng"]
    pt = torch.zeros((6, 1 + 2 * ng, tg["pitch"]), dtype=torch.float64, device=dev)
    pt[:, ng, ng:ng + npair] = torch.from_numpy(samples.T.copy()).to(dev)
    qt = torch.zeros((5,) + pt.shape[1:], dtype=torch.float64, device=dev)
    grhd.prim2con(tg, eos, {}, pt, qt)
    qi = qt[:, ng, ng:ng + npair]
    X, y = grhd.recovery_features(qi, pt[4, ng, ng:ng + npair])
    xm, xs = X.mean(dim=0), X.std(dim=0)
    ym, ys = y.mean(), y.std()
    scal = torch.cat([xm, xs, ym.view(1), ys.view(1)]).float().contiguous()
    Xs = ((X - xm) / xs).float().contiguous()
    ts = ((y - ym) / ys).float().contiguous()
    net = grhd.MLP(grhd.mlp_init(seed), scal)
    gen = torch.Generator(device=dev).manual_seed(seed)
    batch = 8192
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(train_steps):
        idx = torch.randint(0, npair, (batch,), device=dev, generator=gen)
        lr = 2e-3 * 0.5 * (1.0 + math.cos(math.pi * it / train_steps)) + 1e-5
        net.train_step(Xs[idx].contiguous(), ts[idx].contiguous(), lr)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    _, full_loss = grhd.mlp_grad(net.params, Xs, ts)
    return net, {"pairs": npair, "steps": train_steps, "batch": batch, "seconds": train_s,
                 "mse_standardised": float(full_loss.cpu()[0])}


def combined_form(args, grid, eos, metric, metric_np, make_state, value_fp64, Stepper):
    """The headline star in mixed precision with and without the learned
    recovery guess: through a one-patch batched plan (the whole substep --
    recovery, stage kernel, fold -- one graph launch) and through the
    chained stage (one kernel per substep)."""
    import torch

    import synth
    from paper_2502_03223_amd import grhd
    dev = torch.device("cuda:0")
    nzone = grid["nx"] * grid["nz"]
    dt = 0.4 * grid["dx"]
    c2p = dict(w_max=100.0, rho_atm=1e-10)
    net, train_rec = train_guess(synth.star_recovery_samples(4321, args.train_pairs), eos, 2,
                                 max(args.train_steps // 4, 100), dev)
    roles = [("q", "q", "q1"), ("q", "q1", "q2"), ("q", "q2", "q1")]
    res = {"workload": "the headline star, one-patch plan, SSP-RK3", "train": train_rec}

    def descr(b, s):
        qn, qs, qo = roles[s]
        return [dict(grid=grid, metric=metric, qn=b[qn], qs=b[qs], qout=b[qo], p=b["p"],
                     stage=dict(grhd.SSPRK3[s], dt=dt), eos_id=0)]

    def make(mlp):
        q = make_state()
        b = dict(q=q, q1=torch.zeros_like(q), q2=torch.zeros_like(q),
                 p=torch.zeros((6,) + q.shape[1:], dtype=torch.float64, device=dev))
        opts = dict(recon="ppm", riemann="hllc", prec="mixed", c2p=dict(c2p, mlp=mlp))
        plan = grhd.Plan(descr(b, 0), [eos], opts)
        b["q"].copy_(make_state())
        swapped = dict(b, q=b["q1"], q1=b["q"])
        tables = [[plan.table(descr(bb, s)) for s in range(3)] for bb in (b, swapped)]
        return plan, b, tables

    for name, mlp in (("mixed_batched", None), ("mixed_batched_learned", net.buf)):
        plan, b, tables = make(mlp)
        diag = grhd.new_diag()
        par = [0]

        def step():
            for s in range(3):
                plan(tables[par[0]][s], diag=diag)
            par[0] ^= 1
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        d = grhd.read_diag(diag)
        v = 3 * nzone * args.steps / wall
        res[name] = {"value": v, "ms_per_step": wall * 1e3 / args.steps, "speedup_vs_fp64": v / value_fp64,
                     "evals_last_stage": d["iter_sum"], "evals_max_last_stage": d["iter_max"]}
        # accuracy: the same number of substeps from the same initial data as
        # the FP64 path (chained FP64 stepper), L1 of the primitives
        if name == "mixed_batched_learned":
            plan.close()
            plan, b, tables = make(mlp)
            par[0] = 0
            nsteps = args.accuracy_substeps // 3
            ref = Stepper("fp64")
            for _ in range(nsteps):
                step()
                ref.step()
            cur = b["q"] if nsteps % 2 == 0 else b["q1"]
            pc = torch.zeros_like(b["p"])
            grhd.con2prim(grid, eos, metric, c2p, cur.clone(), pc)
            res[name]["accuracy_vs_fp64"] = l1_diffs(grid, metric_np, pc, ref.prims())
            res[name]["accuracy_vs_fp64"]["substeps"] = 3 * nsteps
        plan.close()
    res["guess_speedup"] = res["mixed_batched_learned"]["value"] / res["mixed_batched"]["value"]
    # the same with the chained mixed stage (one kernel per substep, the
    # recovery of q_out at its end, seeded by the network or not)
    for name, mlp in (("mixed_chained", None), ("mixed_chained_learned", net.buf)):
        st = Stepper("mixed", True, mlp)
        for _ in range(args.warmup):
            st.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            st.step()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        d = grhd.read_diag(st.diag)
        v = 3 * nzone * args.steps / wall
        res[name] = {"value": v, "ms_per_step": wall * 1e3 / args.steps, "speedup_vs_fp64": v / value_fp64,
                     "evals_last_stage": d["iter_sum"], "evals_max_last_stage": d["iter_max"]}
        if mlp is not None:
            st = Stepper("mixed", True, mlp)
            ref = Stepper("fp64")
            nsteps = args.accuracy_substeps // 3
            for _ in range(nsteps):
                st.step()
                ref.step()
            res[name]["accuracy_vs_fp64"] = l1_diffs(grid, metric_np, st.prims(), ref.prims())
            res[name]["accuracy_vs_fp64"]["substeps"] = 3 * nsteps
    res["guess_speedup_chained"] = res["mixed_chained_learned"]["value"] / res["mixed_chained"]["value"]
    return res


def l1_diffs(grid, metric_np, pa, pb):
    """L1 differences of two primitive states: rho and eps relative with the
    sqrt(-g) x weight, v^varpi + v^z absolute and x weighted."""
    import synth
    P = synth.interior(grid, pa.cpu().numpy())
    R = synth.interior(grid, pb.cpu().numpy())
    X, _ = synth.cell_coords(grid)
    x = synth.interior(grid, X)
    Wm = synth.interior(grid, metric_np["W"])
    alp = synth.interior(grid, metric_np["alp"])
    wgt = alp * Wm ** -3 * x

    def l1rel(a, b):
        return float((np.abs(a - b) * wgt).sum() / (np.abs(b) * wgt).sum())

    def vel(Q):
        w = np.sqrt(1.0 + Wm ** 2 * (Q[1] ** 2 + Q[2] ** 2 + Q[3] ** 2))
        return Wm ** 2 * Q[1] / w, Wm ** 2 * Q[3] / w
    vx, vz = vel(P)
    rx, rz = vel(R)
    return dict(l1_rel_rho=l1rel(P[0], R[0]), l1_rel_eps=l1rel(P[5], R[5]),
                l1_abs_v=float(((np.abs(vx - rx) + np.abs(vz - rz)) * x).sum() / x.sum()),
                max_abs_v_fp64=float(np.abs(np.stack([rx, rz])).max()))


def batched_form(args, tov):
    """Six nested 256^2 star levels plus 64 thin Riemann patches: one
    batched graph launch per substep against one library call per patch."""
    import torch

    import synth
    from paper_2502_03223_amd import grhd
    dev = torch.device("cuda:0")
    patches = []
    for lvl, g in enumerate(synth.fmr_levels(6, 256, finest_extent=20.0)):
        p, met, _ = synth.star_problem(g, seed=100 + lvl, tov=tov)
        patches.append(dict(grid=g, metric={k: torch.from_numpy(v).to(dev) for k, v in met.items()},
                            p0=p, eos_id=0))
    gam = 5.0 / 3.0
    sizes = synth.riemann_patch_sizes(7, 64, 128, 2048)
    for nxr, (L, R) in zip(sizes, synth.riemann_states(7, 64, gam)):
        g = synth.riemann_grid(nxr, nz=8)
        patches.append(dict(grid=g, metric={}, p0=synth.riemann_prims(g, L, R, gam), eos_id=1))
    eos_table = [synth.ideal_eos(tov["G"], K=tov["K"]), synth.ideal_eos(gam)]
    zones = sum(pt["grid"]["nx"] * pt["grid"]["nz"] for pt in patches)
    c2p = dict(w_max=100.0, rho_atm=1e-10)

    def alloc():
        bufs = []
        for pt in patches:
            p = torch.from_numpy(pt["p0"]).to(dev)
            q = torch.zeros((5,) + p.shape[1:], dtype=torch.float64, device=dev)
            grhd.prim2con(pt["grid"], eos_table[pt["eos_id"]], pt["metric"], p, q, with_ghosts=True)
            bufs.append(dict(q=q, q1=torch.zeros_like(q), q2=torch.zeros_like(q), p=p.clone()))
        return bufs

    def descr(b, pt, s, qn, qs, qo):
        return dict(grid=pt["grid"], metric=pt["metric"], qn=b[qn], qs=b[qs], qout=b[qo], p=b["p"],
                    stage=dict(grhd.SSPRK3[s], dt=0.4 * pt["grid"]["dx"]), eos_id=pt["eos_id"])
    roles = [("q", "q", "q1"), ("q", "q1", "q2"), ("q", "q2", "q1")]
    res = {"zones": zones, "patches": len(patches),
           "workload": "6 nested 256^2 TOV star levels (outer edges 20..640) + 64 Riemann patches "
                       "N_x log-uniform [128, 2048] x 8 periodic z, Gamma 5/3; SSP-RK3"}
    steps = max(args.steps // 2, 5)
    for prec in ("mixed", "fp64"):
        opts = dict(recon="ppm", riemann="hllc", prec=prec, c2p=c2p)
        A = alloc()
        plan = grhd.Plan([descr(b, pt, 0, *roles[0]) for b, pt in zip(A, patches)], eos_table, opts)
        A = alloc()
        diag = grhd.new_diag()
        # marshalled once: step parity (q and q1 swap every step) x stage
        swapped = [dict(b, q=b["q1"], q1=b["q"]) for b in A]
        tables = [[plan.table([descr(b, pt, s, *roles[s]) for b, pt in zip(bufs, patches)])
                   for s in range(3)] for bufs in (A, swapped)]
        par = [0]

        def step_batched():
            for s in range(3):
                plan(tables[par[0]][s], diag=diag)
            par[0] ^= 1
        B = alloc()
        subs = [grhd.Substep(pt["grid"], eos_table[pt["eos_id"]], pt["metric"], opts) for pt in patches]
        dg = grhd.new_diag()
        calls = []
        for bufs in (B, [dict(b, q=b["q1"], q1=b["q"]) for b in B]):
            per = []
            for s in range(3):
                qn, qs, qo = roles[s]
                per.append([sub.bind(dict(grhd.SSPRK3[s], dt=0.4 * pt["grid"]["dx"]), b[qn], b[qs],
                                     b[qo], b["p"], diag=dg) for b, sub, pt in zip(bufs, subs, patches)])
            calls.append(per)
        parb = [0]

        def step_loop():
            for s in range(3):
                for c in calls[parb[0]][s]:
                    c()
            parb[0] ^= 1
        out = {}
        for name, fn in (("batched", step_batched), ("per_patch_calls", step_loop)):
            for _ in range(10):  # first launches of a plan's graph carry one-time costs
                fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                fn()
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            out[name] = 3 * zones * steps / wall
        res[prec] = {"value": out["batched"], "per_patch_calls_value": out["per_patch_calls"],
                     "speedup_vs_per_patch": out["batched"] / out["per_patch_calls"],
                     "tiles": plan.tiles()}
        plan.close()
    return res


def fmr_form(args, tov):
    """Six nested 256^2 levels of the star as one refinement hierarchy
    (level l covers [0, 20 2^(5-l)]^2): zone-updates/s over whole coarse
    steps, counting every level's substeps."""
    import torch

    import synth
    from paper_2502_03223_amd import grhd
    dev = torch.device("cuda:0")
    eos = synth.ideal_eos(tov["G"], K=tov["K"])
    opts = dict(recon="ppm", riemann="hllc", prec="fp64", c2p=dict(w_max=100.0, rho_atm=1e-10))
    res = {"workload": "6 nested 256^2 TOV star levels, outer edges 20..640, cylindrical, "
                       "Berger-Oliger with prolongation, restriction and refluxing; SSP-RK3; "
                       "halo schedule (l_fix 0 and 5) and the (4+4) buffer schedule (l_fix 0); "
                       "zone-updates count own cells"}
    steps = max(args.steps // 10, 3)

    def own(g, nbuf):
        return dict(g, nx=g["nx"] - nbuf, nz=g["nz"] - nbuf)

    def mass(levels, grids):
        M = 0.0
        for l, L in enumerate(levels):
            g = own(grids[l], L["nbuf"])
            q = synth.interior(g, L["q"].cpu().numpy())
            X, _ = synth.cell_coords(g)
            x = synth.interior(g, X)
            dV = 2.0 * math.pi * x * g["dx"] * g["dz"]
            mask = np.ones_like(x, dtype=bool)
            if l + 1 < len(levels):
                co = own(grids[l + 1], levels[l + 1]["nbuf"])
                mask[:co["nz"] // 2, :co["nx"] // 2] = False
            M += float((q[0] * dV)[mask].sum())
        return M
    for key, l_fix, nbuf in (("l_fix_0", 0, 0), ("l_fix_5", 5, 0), ("buffer_l_fix_0", 0, 4)):
        grids = synth.fmr_grids(6, 256, 640.0, geom="cyl", outer="outflow", nbuf=nbuf)
        levels = []
        for lvl, g in enumerate(grids):
            p, met, _ = synth.star_problem(g, seed=100 + lvl, tov=tov)
            metric = {k: torch.from_numpy(v).to(dev) for k, v in met.items()}
            q = torch.zeros((5,) + p.shape[1:], dtype=torch.float64, device=dev)
            grhd.prim2con(g, eos, metric, torch.from_numpy(p).to(dev), q, with_ghosts=True)
            levels.append(dict(grid=g, metric=metric, q=q, nbuf=nbuf if lvl > 0 else 0))
        h = grhd.Hierarchy(levels, eos, opts, l_fix=l_fix)
        # the finest level keeps a Courant factor of 0.4
        dt0 = 0.4 * grids[0]["dx"] / 2 ** min(l_fix, len(grids) - 1)
        level_steps = [1]
        for l in range(1, len(grids)):
            level_steps.append(level_steps[-1] * (1 if l <= l_fix else 2))
        zu = 3 * sum((g["nx"] - L["nbuf"]) * (g["nz"] - L["nbuf"]) * n
                     for g, L, n in zip(grids, levels, level_steps))
        for _ in range(2):
            h.step(dt0)
        torch.cuda.synchronize()
        M0 = mass(levels, grids)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        for _ in range(steps):
            h.step(dt0)
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        M1 = mass(levels, grids)
        res[key] = {"value": zu * steps / wall, "unit": "zone-updates/s",
                    "coarse_steps": steps, "level_steps_per_coarse_step": level_steps,
                    "ms_per_coarse_step": wall * 1e3 / steps,
                    "gpu_ms_per_coarse_step": e0.elapsed_time(e1) / steps,
                    "mass_rel_change": (M1 - M0) / M0}
        h.close()
    return res


def bondi_form(args):
    """Bondi flow on the trumpet slice (general-metric path), held within
    r < 0.4M, exact flow in the outer ghosts; SSP-RK3 to t = 20M."""
    import torch

    import synth
    from paper_2502_03223_amd import grhd
    dev = torch.device("cuda:0")
    c2p = dict(w_max=100.0, rho_atm=1e-14)
    res = {"workload": "Bondi accretion, maximal trumpet slice of Schwarzschild, Gamma 4/3, K = 1, "
                       "r_c = 8M, [0, 16M]^2 cylindrical, fixed for r < 0.4M, SSP-RK3 to t = 20M; "
                       "keys recon[_riemann][_eos]_N (_eos: face eps from the EOS)"}
    errs = {}
    cases = [("ppm", "hllc", "recon"), ("ppm3", "hllc", "recon"), ("ppm3", "tvdlf", "recon"),
             ("minmod", "hllc", "recon"), ("ppm", "hllc", "eos"), ("ppm3", "hllc", "eos")]

    def key_of(recon, riemann, face):
        return recon + ("" if riemann == "hllc" else "_" + riemann) + ("" if face == "recon" else "_eos")
    for (recon, riemann, face), n in [(c, n) for c in cases for n in (64, 128, 256)]:
        d = 16.0 / n
        g = synth.make_grid(n, n, 0.0, 0.0, d, d, "cyl", ("axis", "external", "reflect", "external"))
        p, m, eos, frozen = synth.bondi_problem(g)
        md = {k: torch.from_numpy(v).to(dev) for k, v in m.items()}
        pd = torch.from_numpy(p).to(dev)
        q = torch.zeros((5,) + p.shape[1:], dtype=torch.float64, device=dev)
        grhd.prim2con(g, eos, md, pd, q, with_ghosts=True)
        qfix, q1, q2 = q.clone(), q.clone(), q.clone()
        mask = torch.from_numpy(frozen.astype(np.uint8)).to(dev)
        # the inner region is held inside each stage (no separate pass)
        sub = grhd.Substep(g, eos, md, dict(recon=recon, riemann=riemann, prec="fp64", c2p=c2p,
                                            face_eps=face, fix=(mask, qfix)))
        pw = torch.zeros_like(pd)
        dt = 0.4 * d
        nsteps = int(round(20.0 / dt))
        calls = [sub.bind(dict(grhd.SSPRK3[s], dt=dt), qn, qs, qo, pw)
                 for s, (qn, qs, qo) in enumerate([(q, q, q1), (q, q1, q2), (q, q2, q)])]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(nsteps):
            for c in calls:
                c()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        grhd.con2prim(g, eos, md, c2p, q.clone(), pw)
        rho = synth.interior(g, pw.cpu().numpy()[0])
        rho0 = synth.interior(g, p[0])
        X, _ = synth.cell_coords(g)
        x = synth.interior(g, X)
        sg = synth.interior(g, m["alp"] * m["W"] ** -3) * x
        key = key_of(recon, riemann, face)
        errs[(key, n)] = float((np.abs(rho - rho0) * sg).sum() / (np.abs(rho0) * sg).sum())
        res["%s_N%d" % (key, n)] = {"value": 3 * n * n * nsteps / wall, "unit": "zone-updates/s",
                                    "steps": nsteps, "ms_per_step": wall * 1e3 / nsteps,
                                    "l1_rho": errs[(key, n)]}
    for recon, riemann, face in cases:
        key = key_of(recon, riemann, face)
        res["%s_order_64_128" % key] = math.log2(errs[(key, 64)] / errs[(key, 128)])
        res["%s_order_128_256" % key] = math.log2(errs[(key, 128)] / errs[(key, 256)])
    return res


def general_form(args):
    """The general-metric stage at 1024^2 (FP64, recovery pass + stage
    kernel): the Bondi flow on the trumpet slice (lapse, two shift
    components, W and four curvature components as arrays; inner region
    held inside the stage) and a smooth state on a metric with all 17
    fields as arrays (Cartesian, periodic).  Throughput over SSP-RK3 steps
    and the stage kernel's duration (HIP events); the roofline counts the
    bytes one fused pass must move: q_s read and q_out written (40 B each),
    q^n read in stages 2 and 3 (40 B), 8 B per metric array."""
    import torch

    import synth
    from paper_2502_03223_amd import grhd
    dev = torch.device("cuda:0")
    n = 1024
    res = {"workload": "general-metric stage at 1024^2, FP64, SSP-RK3: Bondi on the trumpet slice "
                       "[0, 16M]^2 (8 metric arrays) and a smooth state on a 17-array metric"}
    cases = {}
    d = 16.0 / n
    g = synth.make_grid(n, n, 0.0, 0.0, d, d, "cyl", ("axis", "external", "reflect", "external"))
    p, m, eos, frozen = synth.bondi_problem(g)
    cases["bondi"] = (g, p, m, eos, frozen, dict(w_max=100.0, rho_atm=1e-14))
    g2 = synth.make_grid(n, n, 0.0, 0.0, 1.0 / n, 1.0 / n, "cart", ("periodic",) * 4)
    m2 = synth.general_metric(g2, 7, amp=0.05)
    cases["metric17"] = (g2, synth.smooth_state(g2, 8, vamp=0.3), m2, synth.ideal_eos(5.0 / 3.0), None,
                         dict(w_max=100.0, rho_atm=1e-12))
    steps = max(args.steps, 5)
    for name, (g, p, m, eos, frozen, c2p) in cases.items():
        md = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in m.items()}
        pd = torch.from_numpy(np.ascontiguousarray(p)).to(dev)
        q = torch.zeros((5,) + p.shape[1:], dtype=torch.float64, device=dev)
        grhd.prim2con(g, eos, md, pd, q, with_ghosts=True)
        qfix, q1, q2 = q.clone(), q.clone(), q.clone()
        opts = dict(recon="ppm", riemann="hllc", prec="fp64", c2p=c2p)
        if frozen is not None:
            opts["fix"] = (torch.from_numpy(frozen.astype(np.uint8)).to(dev), qfix)
        sub = grhd.Substep(g, eos, md, opts)
        pw = torch.zeros_like(pd)
        fl = torch.zeros(p.shape[1:], dtype=torch.uint8, device=dev)
        dt = 0.4 * min(g["dx"], g["dz"])
        bufs = [(q, q, q1), (q, q1, q2), (q, q2, q)]
        stages = [grhd.make_stage(dict(s, dt=dt)) for s in grhd.SSPRK3]

        def step(kev=None):
            for s, (qn, qs, qo) in enumerate(bufs):
                sub(stages[s], qn, qs, qo, pw, flags=fl, events=kev[s] if kev else None)
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kevs = [[(grhd.Event(), grhd.Event()) for _ in range(3)] for _ in range(steps)]
        for k in range(steps):
            step(kevs[k])
        torch.cuda.synchronize()
        kms = np.array([[kevs[k][s][0].elapsed_ms(kevs[k][s][1]) for s in range(3)] for k in range(steps)])
        kms = kms.mean(axis=0)
        nzone = g["nx"] * g["nz"]
        narr = len(m)
        per_stage = [8.0 * (10 + narr), 8.0 * (15 + narr), 8.0 * (15 + narr)]
        achieved = float(np.mean(per_stage)) * nzone / (float(kms.mean()) * 1e-3) / 1e9
        res[name] = {"value": 3 * nzone * steps / wall, "unit": "zone-updates/s",
                     "ms_per_step": wall * 1e3 / steps, "kernel_ms": kms.tolist(), "metric_arrays": narr,
                     "bytes_per_zone": per_stage,
                     "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": achieved / HBM_PEAK_GBS}}
    return res


def density_tv(grid, rho):
    """Area-weighted total variation of rho over the interior (cylindrical
    faces: x-faces weighted by their x, z-faces by the cell x)."""
    x = grid["x0"] + (np.arange(grid["nx"]) + 0.5) * grid["dx"]
    xf = grid["x0"] + np.arange(1, grid["nx"]) * grid["dx"]
    tvx = (np.abs(np.diff(rho, axis=1)) * xf[None, :]).sum() * grid["dz"]
    tvz = (np.abs(np.diff(rho, axis=0)) * x[None, :]).sum() * grid["dx"]
    return float(tvx + tvz)


def run_bondi(grid, p, m, eos, frozen, opts, t_end):
    """SSP-RK3 of a Bondi-type state with the inner region held; returns
    (final primitives, zone-updates/s)."""
    import torch

    from paper_2502_03223_amd import grhd
    dev = torch.device("cuda:0")
    md = {k: torch.from_numpy(v).to(dev) for k, v in m.items()}
    pd = torch.from_numpy(p).to(dev)
    q = torch.zeros((5,) + p.shape[1:], dtype=torch.float64, device=dev)
    grhd.prim2con(grid, eos, md, pd, q, with_ghosts=True)
    qfix, q1, q2 = q.clone(), q.clone(), q.clone()
    mask = torch.from_numpy(frozen.astype(np.uint8)).to(dev)
    sub = grhd.Substep(grid, eos, md, dict(opts, fix=(mask, qfix)))
    pw = torch.zeros_like(pd)
    dt = 0.4 * grid["dx"]
    nsteps = int(round(t_end / dt))
    calls = [sub.bind(dict(grhd.SSPRK3[s], dt=dt), qn, qs, qo, pw)
             for s, (qn, qs, qo) in enumerate([(q, q, q1), (q, q1, q2), (q, q2, q)])]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(nsteps):
        for c in calls:
            c()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    grhd.con2prim(grid, eos, md, opts["c2p"], q.clone(), pw)
    return pw.cpu().numpy(), 3 * grid["nx"] * grid["nz"] * nsteps / wall


def bondi_rt_form(args):
    """The paper's hot-bubble test on the Bondi flow: HLLC against TVDLF."""
    import synth
    n = 512
    d = 16.0 / n
    g = synth.make_grid(n, n, 0.0, 0.0, d, d, "cyl", ("axis", "external", "reflect", "external"))
    p, m, eos, frozen = synth.modified_bondi_problem(g)
    res = {"workload": "Bondi flow with a hot bubble (rho x 0.1, P x 50, u = 0 inside r < 3M [1 + 0.05 "
                       "(cos 80 theta + 1)]), 512^2 on [0, 16M]^2, PPM, SSP-RK3 to t = 25M"}
    tv0 = density_tv(g, synth.interior(g, p[0]))
    for riemann in ("hllc", "tvdlf"):
        opts = dict(recon="ppm", riemann=riemann, prec="fp64", c2p=dict(w_max=100.0, rho_atm=1e-14))
        pf, rate = run_bondi(g, p, m, eos, frozen, opts, 25.0)
        res[riemann] = {"value": rate, "unit": "zone-updates/s",
                        "density_tv_over_initial": density_tv(g, synth.interior(g, pf[0])) / tv0}
    res["tv_ratio_hllc_over_tvdlf"] = (res["hllc"]["density_tv_over_initial"]
                                       / res["tvdlf"]["density_tv_over_initial"])
    return res


def learned_form(args):
    """Recovery of a 2048^2 differentially rotating field: Illinois from the
    bracket (the paper's method) against Newton seeded by the matrix-core
    MLP, trained here on GPU from GPU prim->con pairs of an independent
    seed.  Both land on the same root (max relative primitive difference
    reported); time and master-function evaluations per cell are compared."""
    import torch

    import synth
    from paper_2502_03223_amd import grhd
    dev = torch.device("cuda:0")
    eos = synth.ideal_eos(2.0, 100.0)
    c2p = dict(w_max=100.0, rho_atm=1e-12)
    # ---- training pairs: (D, S, tau) -> P through the library's prim->con
    npair = args.train_pairs
    prims = synth.recovery_samples(12345, npair)
    tg = synth.make_grid(npair, 1, 0.0, 0.0, 1.0, 1.0, "cart", ("outflow",) * 4)
    ng = tg["ng"]
    pt = torch.zeros((6, 1 + 2 * ng, tg["pitch"]), dtype=torch.float64, device=dev)
    pt[:, ng, ng:ng + npair] = torch.from_numpy(prims.T.copy()).to(dev)
    qt = torch.zeros((5,) + pt.shape[1:], dtype=torch.float64, device=dev)
    grhd.prim2con(tg, eos, {}, pt, qt)
    qi = qt[:, ng, ng:ng + npair]
    X, y = grhd.recovery_features(qi, pt[4, ng, ng:ng + npair])
    xm, xs = X.mean(dim=0), X.std(dim=0)
    ym, ys = y.mean(), y.std()
    scal = torch.cat([xm, xs, ym.view(1), ys.view(1)]).float().contiguous()
    Xs = ((X - xm) / xs).float().contiguous()
    ts = ((y - ym) / ys).float().contiguous()
    net = grhd.MLP(grhd.mlp_init(1), scal)
    gen = torch.Generator(device=dev).manual_seed(1)
    batch = 8192
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(args.train_steps):
        idx = torch.randint(0, npair, (batch,), device=dev, generator=gen)
        lr = 2e-3 * 0.5 * (1.0 + math.cos(math.pi * it / args.train_steps)) + 1e-5
        net.train_step(Xs[idx].contiguous(), ts[idx].contiguous(), lr)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    _, full_loss = grhd.mlp_grad(net.params, Xs, ts)
    # ---- the recovery workload
    n = args.learned_n
    grid = synth.make_grid(n, n, 0.0, 0.0, 20.0 / n, 20.0 / n, "cart", ("outflow",) * 4)
    p = torch.from_numpy(synth.rotating_field(grid, 7)).to(dev)
    q = torch.zeros((5,) + p.shape[1:], dtype=torch.float64, device=dev)
    grhd.prim2con(grid, eos, {}, p, q)
    res = {"zones": n * n, "train": {"pairs": npair, "steps": args.train_steps, "batch": batch,
                                     "seconds": train_s, "mse_standardised": float(full_loss.cpu()[0])}}
    outs = {}
    for name, mlp in (("illinois", None), ("mlp_newton", net.buf)):
        cp = dict(c2p, mlp=mlp)
        pp = torch.zeros_like(p)
        dg = grhd.new_diag()
        qq = q.clone()
        for _ in range(3):
            qq.copy_(q)
            grhd.con2prim(grid, eos, {}, cp, qq, pp, diag=dg)
        reps = 10
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(reps)]
        for r in range(reps):
            qq.copy_(q)
            evs[r][0].record()
            grhd.con2prim(grid, eos, {}, cp, qq, pp, diag=dg)
            evs[r][1].record()
        torch.cuda.synchronize()
        ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
        d = grhd.read_diag(dg)
        outs[name] = pp.clone()
        res[name] = {"ms": ms, "zones_per_s": n * n / (ms * 1e-3),
                     "evals_mean": d["iter_sum"] / (n * n), "evals_max": d["iter_max"],
                     "n_fail": d["n_fail"], "n_atm": d["n_atm"]}
    a = synth.interior(grid, outs["illinois"])
    b = synth.interior(grid, outs["mlp_newton"])
    rel = (b - a).abs() / a.abs().amax(dim=(1, 2), keepdim=True).clamp_min(1e-300)
    res["max_rel_diff_vs_illinois"] = float(rel.max().cpu())
    res["speedup"] = res["illinois"]["ms"] / res["mlp_newton"]["ms"]
    return res


def _oracle_band(args):
    """Worker: the oracle (FP64 C) on rows [r0, r1) of the star grid as a
    grid of its own, `steps` SSP-RK3 steps; returns (zone-updates, seconds
    of the substep loop)."""
    grid, eos, metric_np, p_np, c2p, dt, r0, r1, steps = args
    import oracle
    ng = grid["ng"]
    band = dict(grid, nz=r1 - r0, z0=grid["z0"] + r0 * grid["dz"],
                bc=(grid["bc"][0], grid["bc"][1], "reflect" if r0 == 0 else "outflow", "outflow"))
    sl = slice(r0, r1 + 2 * ng)
    p = np.ascontiguousarray(p_np[:, sl])
    met = {k: np.ascontiguousarray(v[sl]) for k, v in metric_np.items()}
    q = oracle.prim2con(band, eos, met, p, with_ghosts=True)
    opts = dict(recon="ppm", riemann="hllc", c2p=c2p)
    t0 = time.perf_counter()
    for _ in range(steps):
        qn = q
        qs = q
        for s in [dict(a=0.0, b=1.0, c=1.0), dict(a=0.75, b=0.25, c=0.25),
                  dict(a=1.0 / 3.0, b=2.0 / 3.0, c=2.0 / 3.0)]:
            r = oracle.rk_substep(band, eos, met, opts, dict(s, dt=dt), qn, qs)
            if s["a"] == 0.0:
                qn = r["qs"]
            qs = r["qout"]
        q = qs
    el = time.perf_counter() - t0
    return band["nx"] * band["nz"] * 3 * steps, el


def cpu_baseline(grid, eos, metric_np, p_np, c2p, dt, steps, rows_single, reps=3):
    """The oracle as it is (plain C, one thread per process, gcc -O3
    without fast-math), timed on the host two ways, each the median of
    `reps` runs: (a) the whole star grid cut into one band of rows per core,
    every core running the oracle on its band at the same time (bands are
    independent samples of the workload; the rate is total zone-updates
    over the wall time of the slowest band); (b) one core on the first
    `rows_single` rows.  Cores: the host's, capped at 16 (the host share
    of one GPU).  Substep loops only; set-up excluded."""
    import multiprocessing as mp
    import platform
    import oracle
    oracle.build(force=False)
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    cores = max(1, min(avail, 16))
    model = platform.processor() or ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    nz = grid["nz"]
    edges = [round(i * nz / cores) for i in range(cores + 1)]
    bands = [(grid, eos, metric_np, p_np, c2p, dt, edges[i], edges[i + 1], steps)
             for i in range(cores) if edges[i + 1] > edges[i]]
    ctx = mp.get_context("spawn")
    multi = []
    with ctx.Pool(len(bands)) as pool:
        pool.map(_oracle_band, [b[:-1] + (1,) for b in bands[:len(bands)]])   # import and page in
        for _ in range(reps):
            t0 = time.perf_counter()
            res = pool.map(_oracle_band, bands)
            wall = time.perf_counter() - t0
            zones = sum(r[0] for r in res)
            multi.append((zones / max(r[1] for r in res), zones, wall))
        single = []
        rs = min(rows_single, nz)
        for _ in range(reps):
            z, el = pool.apply(_oracle_band, ((grid, eos, metric_np, p_np, c2p, dt, 0, rs, steps),))
            single.append((z / el, z, el))
    multi.sort()
    single.sort()
    m, s1 = multi[len(multi) // 2], single[len(single) // 2]
    return {"value": m[0], "unit": "zone-updates/s", "cores": len(bands), "kind": "oracle",
            "cpu_model": model,
            "sample": "oracle FP64 C (gcc -O3, no fast-math, one process per core): the %dx%d star grid "
                      "cut into %d bands of rows, each band run as its own grid by one core for %d SSP-RK3 "
                      "steps (3 substeps each), all at once; %d zone-updates per run, median of %d runs "
                      "(%.1f s of wall time)" % (grid["nx"], nz, len(bands), steps, m[1], reps, m[2]),
            "single_core": {"value": s1[0], "unit": "zone-updates/s", "cores": 1,
                            "sample": "the first %d rows, %d SSP-RK3 steps, %d zone-updates, median of %d "
                                      "runs (%.1f s)" % (rs, steps, s1[1], reps, s1[2])}}


if __name__ == "__main__":
    main()
