"""Throughput of the PFASST-SH hot path on one MI355X.

Workload: two-level PFASST on one GPU, fine T255 (384 x 768 Gaussian grid, 5
Gauss-Lobatto nodes) / coarse T127 (192 x 384, 3 nodes), 16 time slices of
dt = 60 s advanced as one batch, seeded synthetic initial state (n^-2 spectra,
balanced 20 m/s solid body).  One timed step is one PFASST block: the
predictor and N_PF = 8 iterations of Algorithm 1 (the batched fine SDC sweep
of all 16 slices, restriction, coarse F and FAS correction, the serial coarse
chain, interpolation of the increments, new initial conditions; the last
iteration stops after its fine sweep), then the fine collocation residual.
"sweeps/s" counts batched fine sweeps (all 16 slices) per second.

The headline block runs the transform stages of both levels in mixed
precision (FP32 by default) and its last two iterations with an FP64 fine level
(the coarse level keeps the mixed precision); the same block in
plain FP64 is timed next to it, and the states of the two are compared after
every iteration (and against serial FP64 SDC on the same time steps, the
collocation solution PFASST converges to).
Iterations are replayed from captured HIP graphs.  Every kernel of every level
is timed in a second pass over the same blocks with direct launches, each
launch by events attached to the kernel itself (its own start and end
timestamps, no launch gap); the roofline line names the kernel with the
largest time per block, against the bound (MFMA or HBM) its algorithmic work
per launch sets.  The standalone batched SH round trip (synthesis + analysis)
is timed as well.  The oracle is timed on the host cores on a bounded sample,
with all threads and with one.

Prints one JSON line.  `--gpus N` with N > 1 is refused: this build runs on
one GPU (time slices are the batch axis).
"""

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "SDC sweeps/s at T255 x16 slices: mixed vs FP64 at <=1e-6 rel err; SHT TFLOP/s"
FINE = (255, 384, 768, 5)
COARSE = (127, 192, 384, 3)
N_TS = 16
MEMBERS = 1
POWER = 2.0
DT = 60.0
SEED = 3
SEEDS = (SEED,)
WORKLOAD = "pfasst_t255_t127_16slices"

# The large-ensemble workload (--workload ensemble): T511 / T255, 32 steps x 4
# members with n^-3 spectra, 4 iterations, FP32 fine transforms throughout.
ENSEMBLE = dict(FINE=(511, 768, 1536, 5), COARSE=(255, 384, 768, 3), N_TS=32, MEMBERS=4,
                POWER=3.0, SEEDS=(500, 501, 502, 503), WORKLOAD="pfasst_t511_t255_32x4_ensemble")


def initial_states(inputs):
    """[members, 3, K] seeded initial states of the workload."""
    return inputs.seeded_batch(FINE[0], SEEDS, POWER)
PEAKS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0 / 3.0}   # dense MFMA TFLOP/s
HBM_PEAK = 8000.0  # GB/s


def npar(T, m, p):
    return (T + 1 - m - p) // 2 + 1 if m + p <= T + 1 else 0


def legendre_flops(T, nlat, ncols):
    """Useful multiply-adds x 2 of one Legendre contraction (all m, both
    parities, northern rings, degrees to T+1) over `ncols` real columns."""
    J = nlat // 2
    deg = sum(npar(T, m, p) for m in range(T + 1) for p in (0, 1))
    return 2.0 * deg * J * ncols


def ring_flops(nlat, nlon, batch, nsig=9):
    """5 N log2 N per complex FFT of length nlon, 9 per ring pair (4 inverse,
    5 forward)."""
    return 5.0 * nlon * math.log2(nlon) * nsig * (nlat // 2) * batch


def rhs_sht_flops(T, nlat, nlon, batch):
    return (legendre_flops(T, nlat, 8 * batch) + legendre_flops(T, nlat, 10 * batch)
            + ring_flops(nlat, nlon, batch))


def block_sht_flops(fine, coarse, n_ts, n_pf, members=1):
    """Algorithmic SHT flops of one PFASST block (predictor + n_pf iterations,
    the last stopping after the fine sweep), counted per RHS evaluation."""
    Tf, nlf, nof, nnf = fine
    Tc, nlc, noc, nnc = coarse
    fr = lambda b: rhs_sht_flops(Tf, nlf, nof, b * members)
    cr = lambda b: rhs_sht_flops(Tc, nlc, noc, b * members)
    f = cr(n_ts)                                                # predictor: coarse F at the IC
    for j in range(n_ts):                                       # wavefront stages
        if j >= 1:
            f += cr(n_ts - j)
        f += (nnc - 1) * cr(n_ts - j)
    f += nnf * fr(n_ts)                                         # fine F at all nodes
    for k in range(n_pf):
        f += (nnf - 1) * fr(n_ts)                               # A
        if k == n_pf - 1:
            break
        f += nnc * cr(n_ts)                                     # B
        f += (n_ts - 1) * cr(1) + n_ts * (nnc - 1) * cr(1)      # C
        f += fr(n_ts)                                           # D
    return f


def ring_bytes(T, nlat, rsz, batch):
    """Algorithmic HBM bytes of one fused ring launch: Fourier coefficients of
    4 fields in (parity form, complex) and of 5 fields out."""
    L, J = T + 1, nlat // 2
    return (4 + 5) * 2 * L * J * batch * 2 * rsz


def sweep_node_bytes(T, nn, B, rsz):
    """Algorithmic HBM bytes of one fused sweep-node launch, averaged over the
    nodes 1..M of a sweep: FP64 states of 3 K complex per slice read and written
    (node 1: Theta^0 and all F to form the old-iterate sums, S_2..S_M written;
    node i: S_i, F of nodes 1..i-1 but F_E of node i-1 (assembled in the same
    kernel from the analysed products of node i-1, which are read) read, F_E of
    node i-1 written), plus Theta^i and F_I^i and the synthesis operand."""
    M = nn - 1
    K = (T + 1) * (T + 2) // 2
    st = 3 * K * 16 * B                                   # one FP64 state array
    Kx = K + T + 1
    y = 5 * Kx * 2 * rsz * B                              # analysed products
    x = 8 * Kx * rsz * B                                  # synthesis operand (4 fields, complex)
    tot = 0
    for i in range(1, M + 1):
        if i == 1:
            tot += (1 + 2 * nn) * st + (M - 1) * st
        else:
            tot += st + (2 * (i - 1) - 1) * st + y + st
        tot += 2 * st + x
    return tot / M


def table_bytes(T, nlat, prec):
    """Bytes of one packed Legendre table (degrees to T+1, northern rings):
    FP64 8 B per value, FP32 4 B, BF16x3 a hi and a lo bf16 (4 B)."""
    deg = sum(npar(T, m, p) for m in range(T + 1) for p in (0, 1))
    return deg * (nlat // 2) * (8 if prec == "fp64" else 4)


def kernel_work(kernel, T, nlat, nlon, nn, b, prec):
    """Algorithmic work of one launch of a profiled kernel at batch b: useful
    MFMA flops and the bytes it must move through HBM (tables, operands in
    and out, FP64 spectral states), None for kernels without a model.  The
    sweep node of a batch of one or two slices on FP64 / FP32 levels is the
    fused per-order kernel (k_node_fused): the analysis of the previous
    node's products, the node update and the synthesis of the new state."""
    rsz = 8 if prec == "fp64" else 4
    L, J = T + 1, nlat // 2
    K = (T + 1) * (T + 2) // 2
    deg = sum(npar(T, m, p) for m in range(T + 1) for p in (0, 1))
    st = 3 * K * 16 * b
    op = {"fp64": "OpF64", "fp32": "OpF32", "bf16x3": "OpBF3"}[prec]
    xs = deg * 8 * b * (4 if prec == "bf16x3" else rsz)           # synthesis operand
    f4 = 4 * 2 * L * J * b * 2 * rsz                                # Fourier coefficients
    g = 5 * 2 * L * J * b * 2 * (8 if prec == "fp64" else 4)        # analysis operand
    y = 5 * (K + T + 1) * b * 2 * rsz                               # analysed products
    if kernel == "leg_synth":
        return {"flops": legendre_flops(T, nlat, 8 * b), "bytes": table_bytes(T, nlat, prec) + xs + f4,
                "symbol": f"k_leg_synth*<{op}>"}
    if kernel == "leg_anal":
        return {"flops": legendre_flops(T, nlat, 10 * b), "bytes": table_bytes(T, nlat, prec) + g + y,
                "symbol": f"k_leg_anal*<{op}>"}
    if kernel == "ring":
        return {"flops": 0.0, "bytes": ring_bytes(T, nlat, rsz, b), "symbol": f"k_ring_rhs<{op}, {nlon}>"}
    if kernel == "prep":
        return {"flops": 0.0, "bytes": 2 * st + xs, "symbol": f"k_prep_rhs<{op}>"}
    if kernel == "assemble":
        return {"flops": 0.0, "bytes": y + st, "symbol": "k_assemble"}
    if kernel == "sweep_node":
        if b <= 2 and prec in ("fp64", "fp32"):
            states = sweep_node_bytes(T, nn, b, rsz) - (y + xs)
            return {"flops": legendre_flops(T, nlat, 8 * b) + legendre_flops(T, nlat, 10 * b),
                    "bytes": 2 * table_bytes(T, nlat, prec) + g + f4 + states,
                    "symbol": f"k_node_fused<{op}, {nn}>"}
        return {"flops": 0.0, "bytes": sweep_node_bytes(T, nn, b, rsz), "symbol": f"k_sweep_step<{op}, {nn}>"}
    return None


def roofline_of(w, avg_s, prec):
    """Roofline of one kernel from its work per launch and average launch
    time: the bound is the resource whose peak needs the longer time for that
    work (MFMA flops at the precision's dense peak, or bytes at 8 TB/s)."""
    t_mfma = w["flops"] / (PEAKS[prec] * 1e12) if w["flops"] else 0.0
    t_hbm = w["bytes"] / (HBM_PEAK * 1e9)
    mf = {"bound": "mfma", "achieved": w["flops"] / avg_s / 1e12, "peak": PEAKS[prec],
          "unit": "TFLOP/s", "work": w["flops"]} if w["flops"] else None
    hb = {"bound": "hbm", "achieved": w["bytes"] / avg_s / 1e9, "peak": HBM_PEAK, "unit": "GB/s",
          "work": w["bytes"]}
    for r in (mf, hb):
        if r:
            r["frac"] = r["achieved"] / r["peak"]
    main, other = (mf, hb) if t_mfma > t_hbm else (hb, mf)
    main["other_bound"] = None if other is None else {k: other[k] for k in ("bound", "achieved", "peak", "unit", "frac")}
    main["algorithmic_time_us"] = max(t_mfma, t_hbm) * 1e6
    return main


TRAFFIC_TABLE = os.path.join(HERE, "profiles", "traffic_per_launch.md")


def source_digest(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(HERE, "paper_1904_05988_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


KERNEL_SOURCES = {"leg_synth": ["k_legendre.hip", "mfma_ops.h", "pfsh_internal.h"],
                  "leg_anal": ["k_legendre.hip", "mfma_ops.h", "pfsh_internal.h"],
                  "ring": ["k_ring.hip", "mfma_ops.h", "pfsh_internal.h"],
                  "prep": ["k_spectral.hip", "mfma_ops.h", "pfsh_internal.h"],
                  "assemble": ["k_spectral.hip", "mfma_ops.h", "pfsh_internal.h"],
                  "sweep_node": ["k_spectral.hip", "mfma_ops.h", "pfsh_internal.h"]}


def measured_traffic(dom):
    """HBM bytes per launch of the dominant kernel from the committed counter
    table (FETCH_SIZE + WRITE_SIZE, scaled by the plain-copy calibration), if
    the table has its (level, kernel, batch) and was taken on the kernel's
    current source; otherwise None and the reason."""
    if not os.path.exists(TRAFFIC_TABLE):
        return None, "no counter table"
    key = f"{dom['level']}/{dom['kernel']}/b{dom['batch']}"
    digest = source_digest(KERNEL_SOURCES[dom["kernel"]])
    with open(TRAFFIC_TABLE) as f:
        for line in f:
            cells = [c.strip() for c in line.strip().strip("|").split("|")]
            if len(cells) >= 5 and cells[0] == f"`{key}`":
                if cells[4].strip("`") != digest:
                    return None, f"counters of {key} taken on another source ({cells[4]})"
                return float(cells[2]) + float(cells[3]), f"{TRAFFIC_TABLE.split(os.sep)[-2]}/traffic_per_launch.md"
    return None, f"no counters for {key}"


def sht_roundtrip_benchmark(torch, pfsh, reps=20, rounds=5):
    """The standalone batched scalar SH round trip at the fine level: 64
    fields (16 slices x 4) of T255 synthesized to the 384 x 768 grid and
    analysed back, FP64 and FP32 transforms; TFLOP/s on the algorithmic
    count 2 (2 K nlat + 2.5 nlat nlon log2 nlon) per field, and the round
    trip's error."""
    Tf, nlf, nof, _ = FINE
    nf = 64
    K = (Tf + 1) * (Tf + 2) // 2
    flops = nf * 2 * (2 * K * nlf + 2.5 * nlf * nof * math.log2(nof))
    g = torch.Generator(device="cuda").manual_seed(7)
    spec = torch.randn((nf, K), dtype=torch.complex128, device="cuda", generator=g)
    spec[:, : Tf + 1] = spec[:, : Tf + 1].real
    out = {}
    for prec in ("fp64", "fp32"):
        gl = pfsh.Level(Tf, nlf, nof, 3, max_batch=nf // 4, precision=prec)
        grid = gl.sh_synthesis(spec)
        back = gl.sh_analysis(grid)
        err = float((back - spec).abs().max() / spec.abs().max())
        times = []
        for _ in range(rounds):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                gl.sh_synthesis(spec, grid)
                gl.sh_analysis(grid, back)
            b.record()
            b.synchronize()
            times.append(a.elapsed_time(b) / reps)
        ms = float(np.median(times))
        out[prec] = {"fields": nf, "ms": ms, "tflops": flops / (ms * 1e-3) / 1e12,
                     "round_trip_rel_err": err}
        gl.close()
    return out


def make_block(args, mixed, n64, pfsh, inputs, torch):
    """Levels, PFASST context, arrays and the block closure for one precision
    recipe: the transforms of both levels in `mixed`, an FP64 fine level for
    the last n64 iterations (--coarse-fp64: the coarse level FP64 throughout;
    --finish-coarse-fp64: FP64 on the coarse level too in those iterations)."""
    dev = torch.device("cuda", 0)
    Tf, nlf, nof, nnf = FINE
    Tc, nlc, noc, nnc = COARSE
    B = N_TS * MEMBERS
    # workspaces for all nodes of all slices at once (F at every node in one call)
    gfm = pfsh.Level(Tf, nlf, nof, nnf, max_batch=B * nnf, precision=mixed)
    gc = pfsh.Level(Tc, nlc, noc, nnc, max_batch=B * nnc)
    # coarse level of the mixed iterations: FP64, or the fine level's precision
    gcm = gc if (mixed == "fp64" or getattr(args, "coarse_fp64", False)) else \
        pfsh.Level(Tc, nlc, noc, nnc, max_batch=B * nnc, precision=mixed)
    gf64 = gfm if (mixed == "fp64" or n64 == 0) else pfsh.Level(Tf, nlf, nof, nnf, max_batch=B)
    pf = pfsh.Pfasst(gfm, gcm, N_TS, MEMBERS)
    th0 = torch.from_numpy(initial_states(inputs)).to(dev)
    thf, fef, fif = gfm.space_time(B), gfm.space_time(B), gfm.space_time(B)
    res = torch.empty((B, 3), dtype=torch.float64, device=dev)
    k_switch = args.n_pf - n64
    # coarse level of the FP64 finishing iterations
    gcf = gc if getattr(args, "finish_coarse_fp64", False) else gcm
    tuned = {}
    if not getattr(args, "no_tune", False):
        # the batches each level runs: fine sweeps of all slices (the wavefront
        # order also smaller groups), coarse batched steps and the serial chain
        fine_b = [B] if args.schedule == "iterations" else sorted({B, 8, 4, 2, 1}, reverse=True)
        coarse_b = sorted({MEMBERS, 2 * MEMBERS, 4 * MEMBERS, 8 * MEMBERS, B} & set(range(1, B + 1)))
        coarse_b.append(B * nnc)
        # The fine levels are tuned with cold caches: in a block the other
        # kernels of a sweep evict the tables between two launches of a stage.
        # The coarse chain runs its stages back to back (hot caches).
        for name, lv, batches in (("fine", gfm, fine_b + [B * nnf]), ("fine_fp64", gf64, fine_b),
                                  ("coarse", gc, coarse_b), ("coarse_mixed", gcm, coarse_b)):
            if (name == "fine_fp64" and gf64 is gfm) or (name == "coarse_mixed" and gcm is gc):
                continue
            tuned[name] = {b: {k: v[0] for k, v in lv.autotune(b, reps=10, cold=name != "coarse").items()}
                           for b in batches}
        torch.cuda.synchronize()

    def block():
        pf.set_levels(gfm, gcm)
        pf.predict(DT, th0, thf, fef, fif)
        if args.schedule == "wavefront":
            pf.run(DT, thf, fef, fif, args.n_pf, fine_alt=None if n64 == 0 else gf64,
                   k_switch=k_switch)
        else:
            for k in range(args.n_pf):
                if k == k_switch:
                    pf.set_levels(gf64, gcf)
                pf.iterate(DT, thf, fef, fif, last=(k == args.n_pf - 1))
        gf64.residual(DT, thf, fef, fif, out=res)

    return dict(block=block, pf=pf, levels=(gfm, gc, gf64, gcm), arrays=(thf, fef, fif), res=res,
                tuned=tuned, finish_coarse=gcf)


def run_gpu(args, mixed, n64, torch, pfsh, inputs, profile=False):
    """K timed PFASST blocks of one precision recipe."""
    ctx = make_block(args, mixed, n64, pfsh, inputs, torch)
    pf, block = ctx["pf"], ctx["block"]
    gfm, gc, gf64, gcm = ctx["levels"]
    named = ([("fine", gfm), ("coarse", gc)] + ([] if gf64 is gfm else [("fine_fp64", gf64)])
             + ([] if gcm is gc else [("coarse_mixed", gcm)]))
    thf, fef, fif = ctx["arrays"]
    stream = torch.cuda.Stream()
    pf.set_graphs(not profile)
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            block()
        torch.cuda.synchronize()
        if profile:
            for _, lv in named:
                lv.profile(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            block()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        per_level = None
        if profile:
            for _, lv in named:
                lv.profile(False)
            # every launch of every level, ms per block (kernel timestamps, no graphs),
            # and the same split by the batch of the launch
            per_level, groups = {}, []
            B = N_TS * MEMBERS
            for name, lv in named:
                d = {k: lv.profile_read(k) for k in lv.KERNELS}
                per_level[name] = {k: round(ms / args.steps, 4) for k, (n, ms) in d.items() if n}
                cand = sorted(set(range(1, B + 1)) | {B * lv.n_nodes})
                for k, (n_all, _) in d.items():
                    if not n_all:
                        continue
                    for b in cand:
                        n, ms = lv.profile_read(k, batch=b)
                        if n:
                            groups.append({"level": name, "kernel": k, "batch": b, "launches": n,
                                           "ms": ms})
            per_level["_groups"] = groups
        s0 = time.perf_counter()
        for _ in range(10):
            gfm.sdc_sweep(DT, thf, fef, fif)
        torch.cuda.synchronize()
        sweep_ms = (time.perf_counter() - s0) * 1e3 / 10
    pf.set_graphs(False)
    pf.close()
    return dict(ms=(t1 - t0) * 1e3 / args.steps, per_level=per_level, sweep_ms=sweep_ms,
                tuned=ctx["tuned"])


def run_states(args, mixed, n64, torch, pfsh, inputs):
    """One block from the seeded state with the iteration schedule (the
    wavefront order gives bitwise the same states); returns the fine last-node
    values of all slices after each iteration."""
    a = argparse.Namespace(**vars(args))
    a.schedule = "iterations"
    a.no_tune = True
    ctx = make_block(a, mixed, n64, pfsh, inputs, torch)
    pf, (gfm, gc, gf64, gcm) = ctx["pf"], ctx["levels"]
    thf, fef, fif = ctx["arrays"]
    th0 = torch.from_numpy(initial_states(inputs)).to("cuda")
    pf.set_levels(gfm, gcm)
    pf.predict(DT, th0, thf, fef, fif)
    out = []
    for k in range(args.n_pf):
        if k == args.n_pf - n64:
            pf.set_levels(gf64, ctx["finish_coarse"])
        pf.iterate(DT, thf, fef, fif, last=(k == args.n_pf - 1))
        out.append(thf[:, -1].cpu().numpy())
    pf.close()
    return out


def serial_reference(torch, pfsh, inputs, nsweeps=20):
    """Serial FP64 SDC on the fine level, step after step (collocation solution
    of every time step of the block, to which PFASST converges)."""
    Tf, nlf, nof, nnf = FINE
    gl = pfsh.Level(Tf, nlf, nof, nnf, max_batch=MEMBERS)
    x = torch.from_numpy(initial_states(inputs)).to("cuda")
    out = []
    for _ in range(N_TS):
        th, fe, fi = gl.space_time(MEMBERS), gl.space_time(MEMBERS), gl.space_time(MEMBERS)
        e, i = gl.rhs(x)
        th[:, 0] = x
        fe[:, 0] = e
        fi[:, 0] = i
        gl.spread(th, fe, fi)
        for _ in range(nsweeps):
            gl.sdc_sweep(DT, th, fe, fi)
        x = th[:, -1].contiguous()
        out.append(x.cpu().numpy())
    return np.concatenate(out)       # [step * members + member]


def comparators(torch, pfsh, inputs, costmodel, block_ms_fp64, x_pfasst_fp64, xref, n_pf):
    """The serial schemes of Sec. 5.5 on the same kernels and time steps as the
    block (FP64): SDC(5, N_S = 8) and MLSDC(5, 3, N_ML = 4, 1/2) over the 16
    steps of dt, timed with HIP events (one run after a warm-up), their end
    states against serial collocation, and the speedups of the FP64 PFASST
    block over them next to the cost model's (which counts operator
    applications, not the batching of the slices on one GPU)."""
    Tf, nlf, nof, nnf = FINE
    Tc, nlc, noc, nnc = COARSE
    x0 = torch.from_numpy(initial_states(inputs)).to("cuda")
    out = {}

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        return a.elapsed_time(b)

    gl = pfsh.Level(Tf, nlf, nof, nnf, max_batch=MEMBERS)
    th, fe, fi = gl.space_time(MEMBERS), gl.space_time(MEMBERS), gl.space_time(MEMBERS)
    ns = 8

    def run_sdc():
        th[:, 0] = x0
        gl.sdc_run(DT, th, fe, fi, N_TS, ns)
    ms = timed(run_sdc)
    end = th[:, 0].cpu().numpy()
    out["sdc"] = {"scheme": f"SDC({nnf},{ns})", "ms": ms, "steps": N_TS,
                  "rel_err_vs_collocation_last_step": rel_err_slices(end, xref[-MEMBERS:])}
    gc = pfsh.Level(Tc, nlc, noc, nnc, max_batch=MEMBERS * nnc)
    pf = pfsh.Pfasst(gl, gc, 1, MEMBERS)
    nml = 4

    def run_ml():
        th[:, 0] = x0
        pf.mlsdc_run(DT, th, fe, fi, N_TS, nml)
    ms = timed(run_ml)
    end = th[:, 0].cpu().numpy()
    out["mlsdc"] = {"scheme": f"MLSDC({nnf},{nnc},{nml},1/2)", "ms": ms, "steps": N_TS,
                    "rel_err_vs_collocation_last_step": rel_err_slices(end, xref[-MEMBERS:])}
    pf.close()
    alpha = (Tc + 1) / (Tf + 1)
    out["pfasst_fp64"] = {"scheme": f"PFASST({N_TS},{nnf},{nnc},{n_pf},1/2)", "ms": block_ms_fp64,
                          "rel_err_vs_collocation_last_step":
                              rel_err_slices(x_pfasst_fp64[-MEMBERS:], xref[-MEMBERS:])}
    out["speedup_vs_sdc"] = {"gpu": out["sdc"]["ms"] / block_ms_fp64,
                             "cost_model": costmodel.speedup_vs_sdc(N_TS, nnf - 1, nnc - 1, n_pf, alpha, ns)}
    out["speedup_vs_mlsdc"] = {"gpu": out["mlsdc"]["ms"] / block_ms_fp64,
                               "cost_model": costmodel.speedup_vs_mlsdc(N_TS, nnf - 1, nnc - 1, n_pf, alpha, nml)}
    return out


def sweep_benchmark(torch, pfsh, inputs, reps=20, rounds=5):
    """The batched fine sweep alone, per transform precision: 16 independent
    seeded states (seeds 300..315, spread initial guess) at the fine level,
    direct launches timed with HIP events (median of `rounds` x `reps` sweeps),
    and each precision's state after one sweep against the FP64 sweep.  The
    FP64 and FP32 levels run again in recurrence mode (no Legendre tables:
    P_n^m evaluated inside the Legendre kernels); table_bytes is the level's
    table memory in each mode."""
    Tf, nlf, nof, nnf = FINE
    B = 16
    x0 = torch.from_numpy(inputs.seeded_batch(Tf, range(300, 300 + B), POWER)).to("cuda")
    out, ref = {}, None
    for prec, leg in (("fp64", "table"), ("fp32", "table"), ("bf16x3", "table"),
                      ("fp64", "recurrence"), ("fp32", "recurrence")):
        gl = pfsh.Level(Tf, nlf, nof, nnf, max_batch=B, precision=prec, legendre=leg)
        th, fe, fi = gl.space_time(B), gl.space_time(B), gl.space_time(B)
        e, i = gl.rhs(x0)
        th[:, 0] = x0
        fe[:, 0] = e
        fi[:, 0] = i
        gl.spread(th, fe, fi)
        gl.sdc_sweep(DT, th, fe, fi)
        one = th[:, -1].cpu().numpy()
        if ref is None:
            ref = one
        times = []
        for _ in range(rounds):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                gl.sdc_sweep(DT, th, fe, fi)
            b.record()
            b.synchronize()
            times.append(a.elapsed_time(b) / reps)
        ms = float(np.median(times))
        sht = 4 * rhs_sht_flops(Tf, nlf, nof, B)
        out[prec if leg == "table" else f"{prec}_recurrence"] = {
            "ms": ms, "sweeps_per_s": 1e3 / ms, "slice_sweeps_per_s": B * 1e3 / ms,
            "sht_tflops": sht / (ms * 1e-3) / 1e12,
            "rel_err_vs_fp64_one_sweep": rel_err_slices(one, ref), "table_bytes": gl.bytes()[0]}
        gl.close()
    return out


GOLDEN = os.path.join(HERE, "tests", "golden", "pfasst_t255_t127_16x8.npz")


def oracle_golden_err(final, golden_path=GOLDEN):
    """Error of a block's final fine last-node states [16, 3, K] against the
    FP64 oracle's block on the same workload (tests/golden, written by
    tests/golden/make_pfasst_t255.py from the oracle alone; a fixed sample of
    spectral slots): per time step and variable max |got - ref| / max |ref| on
    the sample (the mean-geopotential slot out of both maxima, as in rel_err),
    the maximum over steps.  None for another workload."""
    if WORKLOAD != "pfasst_t255_t127_16slices" or not os.path.exists(golden_path):
        return None
    d = np.load(golden_path)
    meta = d["meta"]
    if (tuple(int(x) for x in meta[:10]) != FINE + COARSE + (N_TS, 8) or float(meta[10]) != DT
            or int(meta[11]) != SEED):
        return None
    slots, ref = d["slots"], d["final"]
    got = np.asarray(final)[:, :, slots]
    out = np.zeros(3)
    for n in range(ref.shape[0]):
        for v in range(3):
            den = np.abs(ref[n, v]).copy()
            diff = np.abs(got[n, v] - ref[n, v])
            if v == 0:
                den[slots == 0] = 0.0
                diff[slots == 0] = 0.0
            out[v] = max(out[v], diff.max() / den.max())
    return [float(x) for x in out]


def rel_err_slices(a, b):
    """The paper's normalized max-norm error per variable, each slice (time
    step, member) normalized by its own reference; the maximum over slices."""
    return [float(x) for x in np.max([rel_err(a[s:s + 1], b[s:s + 1]) for s in range(len(a))], axis=0)]


def rel_err(a, b):
    """Normalized max-norm error per variable; for the geopotential the mean
    slot (0,0) (sqrt(2) Phibar) is left out of both maxima."""
    out = []
    for v in range(3):
        ref = b[:, v].copy()
        diff = a[:, v] - b[:, v]
        if v == 0:
            ref[:, 0] = 0.0
            diff[:, 0] = 0.0
        out.append(float(np.abs(diff).max() / np.abs(ref).max()))
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(seconds_all=15.0, seconds_one=10.0):
    """The oracle as it stands, on the host: each slice's share of one PFASST
    iteration (fine sweep, restriction, coarse F and tau, coarse F at node 0
    and coarse sweep, interpolation of the three increments, fine F at node 0),
    for as many slices as fit the time budget, scaled to iterations/s of all
    slices; once with the BLAS threads NumPy has (value) and once with one."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import sdc, swe, transfer
    from paper_1904_05988_amd import inputs
    Tf, nlf, nof, nnf = FINE
    Tc, nlc, noc, nnc = COARSE
    lf, lc = swe.Level(Tf, nlf, nof), swe.Level(Tc, nlc, noc)
    sf, sc = sdc.SDC(nnf), sdc.SDC(nnc)
    x0 = initial_states(inputs)[0]
    nsl = N_TS * MEMBERS

    def run(budget):
        th, fe, fi = sdc.spread(lf, x0, nnf)
        done, wall0, cpu0 = 0, time.perf_counter(), time.process_time()
        while True:
            t, e, i = sdc.sweep(lf, sf, DT, th, fe, fi)
            tc = transfer.restrict(sf, sc, Tf, Tc, t)
            ec = np.array([swe.explicit_rhs(lc, x) for x in tc])
            ic = np.array([swe.implicit_rhs(lc, x) for x in tc])
            tau = transfer.fas_tau(sf, sc, Tf, Tc, DT, e, i, ec, ic)
            ec[0], ic[0] = swe.rhs(lc, tc[0])
            tc2, ec2, ic2 = sdc.sweep(lc, sc, DT, tc, ec, ic, tau)
            t = t + transfer.interpolate(sc, sf, Tc, Tf, tc2 - tc)
            e = e + transfer.interpolate(sc, sf, Tc, Tf, ec2 - ec)
            i = i + transfer.interpolate(sc, sf, Tc, Tf, ic2 - ic)
            e[0], i[0] = swe.rhs(lf, t[0])
            done += 1
            if time.perf_counter() - wall0 > budget or done >= nsl:
                break
        return done, time.perf_counter() - wall0, time.process_time() - cpu0

    blas = [{"api": d.get("internal_api"), "version": d.get("version"),
             "threads": d.get("num_threads")} for d in threadpool_info() if d.get("user_api") == "blas"]
    threads = max([d["threads"] or 1 for d in blas] or [1])
    done, wall, cpu = run(seconds_all)
    with threadpool_limits(limits=1):
        done1, wall1, _ = run(seconds_one)
    sample = (f"{{}} of {nsl} slices' share of one PFASST iteration at T{Tf}/T{Tc} ({{:.1f}} s), "
              f"scaled to all {nsl} slices")
    runs = {"all_threads": {"value": done / (wall * nsl), "unit": "sweeps/s", "cores": threads,
                            "sample": sample.format(done, wall), "cpu_time_over_wall": cpu / wall},
            "single_thread": {"value": done1 / (wall1 * nsl), "unit": "sweeps/s", "cores": 1,
                              "sample": sample.format(done1, wall1)}}
    # the headline figure is the faster of the two settings (NumPy's many small
    # matrix products can run slower on many BLAS threads than on one)
    best = max(runs.values(), key=lambda r: r["value"])
    return {"value": best["value"], "unit": "sweeps/s", "kind": "oracle", "cores": best["cores"],
            "sample": best["sample"], "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0)), "blas": blas, "runs": runs}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed PFASST blocks")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mixed", default="fp32", choices=["fp32", "bf16x3"])
    ap.add_argument("--workload", default="t255", choices=["t255", "ensemble"],
                    help="t255: T255/T127, 16 steps (the headline); ensemble: T511/T255, "
                         "32 steps x 4 members")
    ap.add_argument("--n64", type=int, default=None,
                    help="final PFASST iterations with FP64 fine levels in the mixed block "
                         "(default 2; ensemble 0)")
    ap.add_argument("--n-pf", type=int, default=None,
                    help="PFASST iterations per block (default 8; ensemble 4)")
    ap.add_argument("--schedule", default="iterations", choices=["wavefront", "iterations"],
                    help="order of the PFASST work inside a block (same arithmetic)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--coarse-fp64", action="store_true",
                    help="keep the coarse level in FP64 during the mixed iterations too (by "
                         "default its transforms take the mixed precision until the first FP64 "
                         "iteration)")
    ap.add_argument("--finish-coarse-fp64", action="store_true",
                    help="switch the coarse level to FP64 as well for the last n64 iterations "
                         "(by default it keeps the mixed precision: the block's difference to "
                         "the FP64 block sits in the fine modes above the coarse truncation)")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default transform-kernel variants (no autotuning)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized device buffer 5 times (HBM counter calibration)")
    args = ap.parse_args()
    if args.workload == "ensemble":
        globals().update(ENSEMBLE)
    if args.n_pf is None:
        args.n_pf = 8 if args.workload == "t255" else 4
    if args.n64 is None:
        args.n64 = 2 if args.workload == "t255" else 0
    if args.schedule == "wavefront" and args.finish_coarse_fp64:
        print("--finish-coarse-fp64 needs --schedule iterations (the wavefront run switches "
              "the fine level only)", file=sys.stderr)
        sys.exit(2)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (time slices are its batch axis); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1904_05988_amd import inputs, pfsh
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n * 8, "copies": 5}))
        return
    pfsh.lib()   # fails loudly if the HIP library is not built

    r64 = run_gpu(args, "fp64", 0, torch, pfsh, inputs)
    rmx = run_gpu(args, args.mixed, args.n64, torch, pfsh, inputs)
    # the same timed blocks again with direct launches and per-kernel timestamps
    rpr = run_gpu(args, args.mixed, args.n64, torch, pfsh, inputs, profile=True)
    s64 = run_states(args, "fp64", 0, torch, pfsh, inputs)
    smx = run_states(args, args.mixed, args.n64, torch, pfsh, inputs)
    spure = run_states(args, args.mixed, 0, torch, pfsh, inputs)
    x64, xmx, xpure = s64[-1], smx[-1], spure[-1]
    err = rel_err_slices(xmx, x64)
    err_pure = rel_err_slices(xpure, x64)
    err_iter = [rel_err_slices(a, b) for a, b in zip(smx, s64)]
    err_iter_pure = [rel_err_slices(a, b) for a, b in zip(spure, s64)]
    xref = serial_reference(torch, pfsh, inputs)
    sweeps = sweep_benchmark(torch, pfsh, inputs)
    from paper_1904_05988_amd import costmodel
    comps = comparators(torch, pfsh, inputs, costmodel, r64["ms"], x64, xref, args.n_pf)

    # the kernel with the largest time per block over all levels and batches,
    # and every (level, kernel, batch) group against its own bound
    Tf, nlf, nof, nnf = FINE
    Tc, nlc, noc, nnc = COARSE
    B = N_TS * MEMBERS
    geom = {"fine": (FINE, args.mixed), "fine_fp64": (FINE, "fp64"), "coarse": (COARSE, "fp64"),
            "coarse_mixed": (COARSE, args.mixed)}
    groups = []
    for g in rpr["per_level"].pop("_groups"):
        (T, nlat, nlon, nn), prec = geom[g["level"]]
        w = kernel_work(g["kernel"], T, nlat, nlon, nn, g["batch"], prec)
        if w is None:
            continue
        avg_s = g["ms"] / g["launches"] * 1e-3
        r = roofline_of(w, avg_s, prec)
        r.update({"level": g["level"], "kernel": g["kernel"], "symbol": w["symbol"],
                  "batch": g["batch"], "launches_per_block": g["launches"] / args.steps,
                  "ms_per_block": g["ms"] / args.steps, "avg_us": avg_s * 1e6})
        groups.append(r)
    groups.sort(key=lambda r: -r["ms_per_block"])
    if groups:
        dom = groups[0]
        roof = {k: dom[k] for k in ("bound", "achieved", "peak", "unit", "frac")}
        roof["traffic"], roof["traffic_source"] = measured_traffic(dom)
        roof.update({k: dom[k] for k in ("level", "kernel", "symbol", "batch", "avg_us",
                                         "launches_per_block", "ms_per_block")})
        roof["algorithmic_per_launch"] = dom["work"]
        roof["other_bound"] = dom["other_bound"]
    else:
        roof = {"bound": None, "achieved": None, "peak": None, "unit": None, "frac": None,
                "traffic": None, "note": "no profiled launch"}
    stages = {f"{r['level']}/{r['kernel']}/b{r['batch']}":
              {k: r[k] for k in ("bound", "achieved", "unit", "frac", "avg_us", "ms_per_block")}
              for r in groups[:12]}
    sht_rt = sht_roundtrip_benchmark(torch, pfsh)
    sht = block_sht_flops(FINE, COARSE, N_TS, args.n_pf, MEMBERS)
    value = args.n_pf * 1e3 / rmx["ms"]
    out = {
        "metric": METRIC, "value": value, "unit": "sweeps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": rmx["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": f"{args.mixed}+f64", "data": "synthetic",
        "config": {"workload": WORKLOAD, "fine": f"T{Tf} {nlf}x{nof} {nnf} Lobatto nodes",
                   "coarse": f"T{Tc} {nlc}x{noc} {nnc} nodes", "slices": N_TS,
                   "members": MEMBERS, "spectrum": f"n^-{POWER:g}", "dt_s": DT,
                   "n_pf": args.n_pf, "fp64_final_iterations": args.n64,
                   "schedule": args.schedule,
                   "coarse_precision": "fp64" if args.coarse_fp64 else (
                       f"{args.mixed} then fp64" if args.finish_coarse_fp64 and args.n64 > 0
                       else args.mixed),
                   "step": "one PFASST block: predictor + n_pf iterations, fine residual",
                   "seeds": list(SEEDS), "parallelism": "slices x members as batch, 1 GPU"},
        "roofline": roof,
        "stage_fractions": stages,
        "sht_roundtrip": sht_rt,
        "fp64": {"sweeps_per_s": args.n_pf * 1e3 / r64["ms"], "ms_per_step": r64["ms"],
                 "sweep_only_ms": r64["sweep_ms"],
                 "sht_tflops": sht / (r64["ms"] * 1e-3) / 1e12},
        "mixed_rel_err_vs_fp64": err,
        "mixed_ok": bool(max(err) <= 1e-6),
        "rel_err_vs_oracle_block": None if args.n_pf != 8 else {
            "reference": "FP64 oracle block, tests/golden/pfasst_t255_t127_16x8.npz (sampled slots)",
            "fp64": oracle_golden_err(x64), "mixed": oracle_golden_err(xmx)},
        "mixed_without_fp64_iterations_rel_err": err_pure,
        "mixed_rel_err_per_iteration": err_iter,
        "mixed_without_fp64_iterations_rel_err_per_iteration": err_iter_pure,
        "pfasst_err_vs_serial_collocation": {
            "fp64": rel_err_slices(x64, xref), "mixed": rel_err_slices(xmx, xref),
            "mixed_without_fp64_iterations": rel_err_slices(xpure, xref)},
        "sweep_only_ms": rmx["sweep_ms"],
        "sweep_benchmark": sweeps,
        "comparators": comps,
        "sht_tflops": sht / (rmx["ms"] * 1e-3) / 1e12,
        "kernel_ms_per_step_all_levels": rpr["per_level"],
        "tuned_variants": rmx["tuned"],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
