"""Benchmark: dU proposals/s and accepted-move commit time of FMM-KMC on one MI355X.

Workload: periodic cubic box, 128^3 site lattice (spacing 1), N = 10^6 neutral
+-1 charges on seeded random sites, 26 hop targets per charge (first, second
and third neighbour shells: 26M proposal slots per step), octree depth L = 7,
expansion order p = 12; FP64 and mixed precision.

A step is one pass of the whole hot path: the energy change of every slot
(propose) and one accepted move (commit: dU recomputed, every fine-level local
expansion, the multipole path on every level and the far field updated).  The
accepted move is a seeded uniform choice among the valid slots that does not
look at dU.  The reported step is driven by the device (selection on the GPU,
the step replayed from a captured HIP graph); the host-driven step (selection
in Python, one accept call per step) is reported beside it, and the per-kernel
times come from that run.  Inputs are resident on the GPU before timing starts; the one-time
setup (octree build) is timed separately and not part of a step.

A second workload, batched replicas, runs after it unless --skip-batch: 256
independent periodic systems with N_r log-uniform in [1000, 65536] at 50 %
lattice occupancy, 6 hops, p = 10, advanced together (one launch per phase of a
step over all replicas, the step replayed from a captured HIP graph), in mixed
precision and FP64, beside the plain FP64 path (one replica at a time).

Prints one JSON line.  Options: --steps K --warmup W --gpus 1 [--skip-cpu]
[--skip-batch] [--batch-only] [--precision fp64|mixed|both] [--copy-calibration]
[--quick] (a small periodic system for a smoke run).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, published
FP64_PEAK_TFLOPS = 78.6    # MI355X FP64 vector, published
FP32_PEAK_TFLOPS = 157.3
P2L_FLOP = 850             # one P2L of a point charge at p = 12 (irregular recurrences + accumulation)
PROFILE_DIR = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = {"site_phi_s2": "kernels_propose.hip", "slot_lattice": "kernels_propose.hip",
                  "sweep": "kernels_commit.hip"}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_work(kernel, n, N, K, p, precision, exact_self=False):
    """(bound, algorithmic amount per launch, unit) of the three kernels that
    carry a step: what the method must move (bytes) or compute (flop) once."""
    nt = (p + 1) ** 2
    sites = n ** 3
    cells = sites // 8
    mixed = precision == "mixed"
    if kernel == "site_phi_s2":
        # local expansions once (FP32 shadow + FP64 L_0^0 in mixed), charges, occupancy ranks,
        # far-field tables, potentials out (per site and per charge)
        psi = cells * nt * (4 if mixed else 8) + (cells * 8 if mixed else 0)
        return "hbm", psi + sites * ((4 if mixed else 8) + 4 + 8) + N * 8 + n * n * (p + 1) * 8, "B"
    if kernel == "slot_lattice":
        # per slot: dU out, mask out, F in (not with the exact self-image option: a per-hop
        # table); per charge: site, index, q, phi_occ; potential of every site once
        return "hbm", N * K * (8 + 1 + (0 if exact_self else 8)) + N * (4 + 4 + 8 + 8) + sites * 8, "B"
    if kernel == "sweep":
        # 27 copies x 2 endpoints of P2L into every fine cell
        return "alu", cells * 54 * P2L_FLOP, "flop"
    raise KeyError(kernel)


def sweep_bytes(n, p, precision):
    nt = (p + 1) ** 2
    cells = n ** 3 // 8
    return 2 * cells * nt * 8 + (cells * nt * 4 if precision == "mixed" else 0)


def source_sha(kernel):
    import hashlib
    path = os.path.join(ROOT, "paper_1905_04065_amd", "csrc", KERNEL_SOURCES[kernel])
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def profiled_traffic(workload_tag, precision):
    """HBM bytes per launch from the committed rocprofv3 counter summary, per
    kernel, scaled by the copy-kernel calibration; a kernel whose source changed
    since the counters were taken gets None."""
    path = os.path.join(PROFILE_DIR, f"traffic_{workload_tag}.txt")
    out = {}
    if not os.path.exists(path):
        return out
    cal = {}
    rows = []
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            kv = dict(tok.split("=", 1) for tok in line.split()[1:] if "=" in tok)
            if line.startswith("calibration"):
                cal = {k: float(v) for k, v in kv.items()}
            elif line.startswith("kernel"):
                rows.append(kv)
    for kv in rows:
        if kv.get("precision") != precision:
            continue
        name = kv["name"]
        if name not in KERNEL_SOURCES or kv.get("source_sha") != source_sha(name):
            out[name] = None
            continue
        fetch = float(kv["fetch_kib"]) * 1024 * cal.get("fetch_factor", 1.0)
        write = float(kv["write_kib"]) * 1024 * cal.get("write_factor", 1.0)
        out[name] = fetch + write
    return out


def copy_bandwidth(nbytes=1 << 30, reps=5):
    """Device-to-device copy of nbytes (read + write), GB/s of bytes moved."""
    import torch
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    return 2 * nbytes / (ms / 1e3) / 1e9


def run_gpu(precision, n, N, L, p, hops, steps, warmup, seed, self_image="expansion", host_loop=True,
            per_level=False):
    import torch

    from paper_1905_04065_amd import Context

    sites, xyz, q = W.lattice_charges(n, N, seed)
    K = len(hops)
    log(f"[{precision}, self image {self_image}, per-level {per_level}] create n={n} N={N} L={L} p={p} K={K}")
    t0 = time.perf_counter()
    ctx = Context(xyz, q, a=float(n), levels=L, order=p, bc="periodic", precision=precision, lattice_n=n,
                  device=0, self_image=self_image, per_level=per_level)
    U0 = ctx.initialise()
    dU, mask = ctx.propose_lattice(hops)  # builds the per-charge hop table once
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"[{precision}] setup {setup_s:.2f} s, U0 = {U0:.6f}")
    occ = np.zeros(n ** 3, bool)
    occ[sites] = True
    cur = sites.copy()
    rng = np.random.default_rng(seed + 1)

    def choose():
        while True:
            i = int(rng.integers(N))
            k = int(rng.integers(K))
            s = cur[i]
            ijk = np.array([s // (n * n), (s // n) % n, s % n]) + hops[k]
            ijk %= n
            t = (ijk[0] * n + ijk[1]) * n + ijk[2]
            if not occ[t]:
                return i, t

    def step():
        ctx.propose_lattice(hops, dU=dU, mask=mask)
        i, t = choose()
        d = ctx.accept(i, W.site_xyz([t], n)[0])
        occ[cur[i]] = False
        occ[t] = True
        cur[i] = t
        return d

    names = ["site_phi_s2", "site_phi", "slot_lattice", "sweep", "path", "far_refresh", "cheb_a", "cheb_b", "f_rows",
             "f_row1", "self_hops", "book", "move_dU", "levels", "coarse_s2", "coarse_sites"]
    # f_row1 runs on the side stream, beside the sweep
    ktimes, wall, propose_wall, commit_wall = {}, float("nan"), float("nan"), float("nan")
    if host_loop:
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        ctx.set_profiling(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ktimes = {nm: ctx.kernel_time(nm) for nm in names}
        ctx.set_profiling(False)
        # propose-only timing (no commit) for the proposal rate
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.propose_lattice(hops, dU=dU, mask=mask)
        torch.cuda.synchronize()
        propose_wall = time.perf_counter() - t0
        # commit-only timing
        t0 = time.perf_counter()
        for _ in range(steps):
            i, t = choose()
            ctx.accept(i, W.site_xyz([t], n)[0])
            occ[cur[i]] = False
            occ[t] = True
            cur[i] = t
        torch.cuda.synchronize()
        commit_wall = time.perf_counter() - t0
    valid = int(mask.sum().item())
    # the same step driven by the device: selection on the GPU (a seeded uniform
    # choice among the valid slots, as above) and the whole step replayed from a
    # captured HIP graph (a batch of one system), tile sizes autotuned
    from paper_1905_04065_amd import Batch
    b = Batch([ctx], hops)
    tuning = b.tune(rounds=3)
    b.step(rng.random((warmup, 1)))
    u = rng.random((steps, 1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(u)
    torch.cuda.synchronize()
    graph_wall = time.perf_counter() - t0
    b.close()
    ctx.close()
    return dict(setup_s=setup_s, host_ms_per_step=1e3 * wall / steps, ms_per_step=1e3 * graph_wall / steps,
                propose_ms=1e3 * propose_wall / steps, commit_us=1e6 * commit_wall / steps, kernels=ktimes,
                valid_slots=valid, U0=U0, tuning=tuning)


def batch_contexts(precision, p=10, count=256):
    """the replicas of the batched workload: N_r log-uniform in [1000, 65536],
    lattice side n_r = ceil((2 N_r)^(1/3)) (about 50 % occupancy), depth by the
    level rule, periodic, p = 10"""
    from paper_1905_04065_amd import Context
    Ns, ns, Ls = W.replica_sizes(count)
    ctxs = []
    for r in range(count):
        sites, xyz, q = W.replica_system(r, Ns[r], ns[r])
        c = Context(xyz, q, a=float(ns[r]), levels=int(Ls[r]), order=p, bc="periodic", precision=precision,
                    lattice_n=int(ns[r]), device=0)
        c.initialise()
        ctxs.append(c)
        if (r + 1) % 64 == 0:
            log(f"[batch] {precision}: {r + 1}/{count} replicas set up")
    return ctxs, Ns, ns


def run_batched(precision, steps, warmup, seed, tune=True, keep=False):
    """config-5 steps of all replicas as one captured graph per step"""
    import torch

    from paper_1905_04065_amd import Batch
    t0 = time.perf_counter()
    ctxs, Ns, ns = batch_contexts(precision)
    b = Batch(ctxs, W.HOPS6)
    setup_s = time.perf_counter() - t0
    info = b.tune(rounds=5) if tune else b.info()
    R = len(ctxs)
    rng = np.random.default_rng(seed)
    b.step(rng.random((warmup, R)))
    u = rng.random((steps, R))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    moved, site, dU = b.step(u)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # per-phase times over a few more steps as plain launches
    b.set_profiling(True)
    b.step(rng.random((3, R)))
    phases = {}
    for name in ["b_site", "b_slot", "b_count", "b_select", "b_move_dU", "b_frow", "b_sweep", "b_path", "b_book",
                 "b_far_refresh", "b_cheb_a", "b_cheb_b", "b_finish"]:
        ms, n = b.kernel_time(name)
        if n:
            phases[name] = ms / n * 1e3
    b.set_profiling(False)
    moved_frac = float((moved.cpu().numpy() >= 0).mean())
    b.close()
    out = dict(ms_per_step=1e3 * wall / steps, slots_per_step=info["slots_per_step"], tuning=info,
               setup_s=setup_s, phase_us=phases, replicas=R, moved_fraction=moved_frac)
    if keep:
        return out, ctxs
    for c in ctxs:
        c.close()
    return out


def run_unbatched_fp64(ctxs, steps, seed):
    """the plain path: each replica stepped through the single-context API
    (proposal pass, selection on the host from the mask, accept), FP64; the
    contexts continue from wherever earlier (batched) steps left them"""
    import torch
    Ns, ns, _ = W.replica_sizes(len(ctxs))
    R = len(ctxs)
    rng = np.random.default_rng(seed)
    bufs = [(torch.empty((c.N, 6), dtype=torch.float64, device="cuda"),
             torch.empty((c.N, 6), dtype=torch.uint8, device="cuda")) for c in ctxs]
    cur = []
    for r, c in enumerate(ctxs):
        xyz = c.positions().cpu().numpy()
        ijk = np.floor(xyz).astype(np.int64)  # unit spacing: site (i+1/2, ...) -> i
        cur.append((ijk[:, 0] * ns[r] + ijk[:, 1]) * ns[r] + ijk[:, 2])

    def one_step(u):
        for r, c in enumerate(ctxs):
            dU, mask = c.propose_lattice(W.HOPS6, dU=bufs[r][0], mask=bufs[r][1])
            m = mask.cpu().numpy().reshape(-1)  # synchronises
            vs = np.flatnonzero(m)
            slot = vs[int(u[r] * len(vs))]
            i, k = divmod(int(slot), 6)
            nr = int(ns[r])
            s = int(cur[r][i])
            ijk = (np.array([s // (nr * nr), (s // nr) % nr, s % nr]) + W.HOPS6[k]) % nr
            t = int((ijk[0] * nr + ijk[1]) * nr + ijk[2])
            c.accept(i, W.site_xyz([t], nr)[0])
            cur[r][i] = t

    one_step(rng.random(R))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one_step(rng.random(R))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    slots = int(sum(c.N for c in ctxs)) * 6
    for c in ctxs:
        c.close()
    return dict(ms_per_step=1e3 * wall / steps, slots_per_step=slots)


def cpu_baseline(n, N, L, p, hops, seed, budget_s=20.0):
    """The oracle (O-fmm, FP64, OpenMP) on the host cores, on a bounded sample:
    all hops of the charges in a 2x2x2 block of fine cells, after the cells
    those proposals touch have been formed (setup excluded on both sides)."""
    import oracle as O

    sites, xyz, q = W.lattice_charges(n, N, seed)
    t0 = time.perf_counter()
    f = O.FmmKmc(xyz, q, float(n), L, p, "periodic", lazy=True)
    setup = time.perf_counter() - t0
    nc = 2 ** (L - 1)
    w = n / nc
    cells = np.floor(xyz / w).astype(int)
    inblock = np.all((cells >= nc // 2) & (cells < nc // 2 + 2), axis=1)
    idx_c = np.nonzero(inblock)[0]
    t, valid = O.lattice_targets(sites[idx_c], n, hops, True)
    idx = np.repeat(idx_c, len(hops))[valid.reshape(-1)]
    tgt = W.site_xyz(t.reshape(-1)[valid.reshape(-1)], n)
    for x in np.concatenate([xyz[idx_c], tgt]):
        f.local(f.fine_cell_of(x))
    t0 = time.perf_counter()
    reps = 0
    while True:
        f.propose(idx, tgt)
        reps += 1
        el = time.perf_counter() - t0
        if el > budget_s / 4 or reps >= 50:
            break
    rate = reps * len(idx) / el
    threads = int(os.environ.get("OMP_NUM_THREADS", 0)) or len(os.sched_getaffinity(0))
    f.close()
    return dict(value=rate, unit="proposals/s", cores=threads, kind="oracle",
                sample=f"{len(idx)} valid slots (all 26 hops of the {len(idx_c)} charges in a 2x2x2 block of fine "
                       f"cells) x {reps} repetitions, FP64 O-fmm with OpenMP; octree upward pass ({setup:.1f} s) and "
                       f"formation of the touched cells' local expansions excluded")


def roofline_entry(kernel, kt, n, N, K, p, precision, copy_gbs, traffic, exact_self=False):
    ms, launches = kt.get(kernel, (0.0, 0))
    if launches == 0:
        return None
    avg_s = ms / launches / 1e3
    bound, amount, unit = kernel_work(kernel, n, N, K, p, precision, exact_self)
    e = {"kernel": kernel, "avg_us": avg_s * 1e6, "launches": launches}
    if bound == "hbm":
        ach = amount / avg_s / 1e9
        e.update(bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS,
                 frac_of_copy=ach / copy_gbs if copy_gbs else None, algorithmic_bytes=amount)
    else:
        ach = amount / avg_s / 1e12
        peak = FP64_PEAK_TFLOPS
        e.update(bound="alu", achieved=ach, peak=peak, unit="TFLOP/s", frac=ach / peak, algorithmic_flop=amount,
                 hbm_bytes=sweep_bytes(n, p, precision),
                 hbm_GBps=sweep_bytes(n, p, precision) / avg_s / 1e9)
    t = traffic.get(kernel) if traffic else None
    e["traffic"] = t
    return e


def run_slab(steps, warmup, seed, precision="fp64", n=128, N=500000, L=7, p=12, ez=0.1):
    """Charges between grounded plates (mirror images, Sec. 2.2.2) in a uniform
    field: N physical charges on the lower half of the n^3 lattice (50 %
    occupancy; the doubled system has the size of the periodic workload), 26
    hops, one accepted move (a charge and its mirror) per step."""
    import torch

    from paper_1905_04065_amd import Slab

    rng = np.random.default_rng(seed)
    half = n // 2
    sites = rng.choice(n * n * half, N, replace=False)
    ijk = np.stack([sites // (n * half), (sites // half) % n, sites % half], 1)
    q = np.where(np.arange(N) < N // 2, 1.0, -1.0)
    rng.shuffle(q)
    hops = W.HOPS26
    K = len(hops)
    log(f"[slab] create n={n} N={N} (doubled {2 * N}) L={L} p={p} K={K}")
    t0 = time.perf_counter()
    s = Slab((ijk + 0.5).astype(np.float64), q, a=float(n), levels=L, order=p, lattice_n=n, ez=ez,
             precision=precision)
    s.initialise()
    dU, mask = s.propose_lattice(hops)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    occ = set(map(tuple, ijk))
    cur = ijk.copy()

    def choose():
        while True:
            i = int(rng.integers(N))
            t = cur[i] + hops[int(rng.integers(K))]
            t[0] %= n
            t[1] %= n
            if 0 <= t[2] < half and tuple(t) not in occ:
                return i, t

    def move(i, t):
        s.accept(i, t + 0.5)
        occ.discard(tuple(cur[i]))
        occ.add(tuple(t))
        cur[i] = t

    def step():
        s.propose_lattice(hops)
        move(*choose())

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    step_ms = 1e3 * (time.perf_counter() - t0) / steps
    t0 = time.perf_counter()
    for _ in range(steps):
        dU, mask = s.propose_lattice(hops)
    torch.cuda.synchronize()
    propose_us = 1e6 * (time.perf_counter() - t0) / steps
    t0 = time.perf_counter()
    for _ in range(steps):
        move(*choose())
    torch.cuda.synchronize()
    commit_us = 1e6 * (time.perf_counter() - t0) / steps
    valid = int(mask.sum().item())
    s.close()
    slots = N * K
    return {"workload": f"slab between grounded plates: N={N} +-1 charges on the lower half of a {n}^3 lattice "
                        f"(doubled by mirror images to {2 * N}), field E_z={ez}, {K} hops, L={L}, p={p}, {precision}, "
                        "one accepted move (charge and mirror) per step, host-driven",
            "proposals_per_s": slots / (step_ms / 1e3), "ms_per_step": step_ms, "slots_per_step": slots,
            "valid_slots": valid, "propose_us": propose_us, "commit_us": commit_us, "setup_s": setup_s}


def batched_summary(args):
    """256 replicas, p = 10, 6 hops, periodic: mixed and FP64 batched (graph
    steps) against the plain FP64 path (one replica at a time, host selection)"""
    seed = W.BASE_SEED + 5
    steps = max(args.steps, 5)
    log("[batch] mixed")
    mixed = run_batched("mixed", steps, args.warmup, seed)
    log("[batch] fp64")
    fp64, ctxs = run_batched("fp64", steps, args.warmup, seed, keep=True)
    log("[batch] fp64 one replica at a time")
    plain = run_unbatched_fp64(ctxs, 2, seed)
    for c in ctxs:
        c.close()
    slots = mixed["slots_per_step"]
    return {
        "workload": f"{mixed['replicas']} periodic replicas, N_r log-uniform in [1000, 65536] (sum {slots // 6}), "
                    "50 % lattice occupancy, 6 hops, p=10, one accepted move per replica per step",
        "slots_per_step": slots,
        "mixed_batched": {"proposals_per_s": slots / (mixed["ms_per_step"] / 1e3), **mixed},
        "fp64_batched": {"proposals_per_s": slots / (fp64["ms_per_step"] / 1e3), **fp64},
        "fp64_one_replica_at_a_time": {"proposals_per_s": slots / (plain["ms_per_step"] / 1e3), **plain},
        "speedup_mixed_batched_vs_plain_fp64": plain["ms_per_step"] / mixed["ms_per_step"],
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="both", choices=["fp64", "mixed", "both"])
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run the 1 GiB device copy used to calibrate rocprofv3 byte counters")
    ap.add_argument("--quick", action="store_true", help="small periodic system (64^3, N=1e5, L=6)")
    ap.add_argument("--skip-batch", action="store_true",
                    help="leave out the batched-replica and grounded-slab workloads")
    ap.add_argument("--batch-only", action="store_true", help="only the batched-replica workload (JSON to stdout)")
    ap.add_argument("--skip-exact-self", action="store_true",
                    help="leave out the runs with the exact self-image option")
    ap.add_argument("--skip-per-level", action="store_true",
                    help="leave out the runs with per-level local expansions")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU decomposition is "
              "described in DESIGN.md but not built", file=sys.stderr)
        sys.exit(2)
    if args.batch_only:
        print(json.dumps(batched_summary(args)), flush=True)
        return
    if args.quick:
        n, N, L, p, hops = 64, 100000, 6, 12, W.HOPS26
    else:
        n, N, L, p, hops = 128, 1000000, 7, 12, W.HOPS26
    tag = f"periodic{n}_N{N}_p{p}"
    seed = W.BASE_SEED + 4
    K = len(hops)
    precs = ["fp64", "mixed"] if args.precision == "both" else [args.precision]
    res = {pr: run_gpu(pr, n, N, L, p, hops, args.steps, args.warmup, seed) for pr in precs}
    res_exact = {} if args.skip_exact_self else {
        pr: run_gpu(pr, n, N, L, p, hops, args.steps, args.warmup, seed, self_image="exact") for pr in precs}
    res_levels = {} if args.skip_per_level else {
        pr: run_gpu(pr, n, N, L, p, hops, args.steps, args.warmup, seed, per_level=True) for pr in precs}
    res_both = {} if (args.skip_per_level or args.skip_exact_self) else {
        pr: run_gpu(pr, n, N, L, p, hops, args.steps, args.warmup, seed, per_level=True, self_image="exact")
        for pr in precs}
    copy_gbs = copy_bandwidth()
    if args.copy_calibration:
        copy_bandwidth(1 << 30, reps=3)
    head_prec = "fp64" if "fp64" in res else precs[0]
    slots = N * K

    def summary(pr, exact=False, levels=False):
        r = (res_both if (levels and exact) else res_levels if levels else res_exact if exact else res)[pr]
        kt = r["kernels"]
        traffic = {} if (exact or levels) else profiled_traffic(tag, pr)
        roof = {k: roofline_entry(k, kt, n, N, K, p, pr, copy_gbs, traffic, exact)
                for k in ("site_phi_s2", "slot_lattice", "sweep")}
        # the kernel that takes the largest share of a step
        dom = max(roof, key=lambda k: roof[k]["avg_us"] if roof[k] else -1)
        return dict(value=slots / (r["ms_per_step"] / 1e3), ms_per_step=r["ms_per_step"],
                    host_driven_ms_per_step=r["host_ms_per_step"], tuning=r["tuning"],
                    valid_per_s=r["valid_slots"] / (r["ms_per_step"] / 1e3),
                    propose_only_per_s=slots / (r["propose_ms"] / 1e3), propose_us=r["propose_ms"] * 1e3,
                    commit_us=r["commit_us"], setup_s=r["setup_s"],
                    kernel_avg_us={k: (v[0] / max(v[1], 1) * 1e3) for k, v in kt.items() if v[1] > 0},
                    dominant=dom, rooflines=roof)

    head = summary(head_prec)
    dom = head["dominant"]
    droof = dict(head["rooflines"][dom])
    out = {
        "metric": "dU proposals/sec at N=1e6, p=12 (FP64 vs mixed); accepted-move commit us",
        "value": head["value"],
        "unit": "proposals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "step_driver": "device: selection on the GPU, step replayed from a captured HIP graph",
        "host_driven_ms_per_step": head["host_driven_ms_per_step"],
        "tuning": head["tuning"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head_prec == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"periodic {n}^3 lattice, N={N} +-1 charges, {K} hops/charge ({slots} slots/step), "
                               f"L={L}, p={p}, one accepted move per step",
                   "global_batch": slots, "parallelism": "single GPU"},
        "valid_proposals_per_s": head["valid_per_s"],
        "valid_slots": res[head_prec]["valid_slots"],
        "propose_only_per_s": head["propose_only_per_s"],
        "propose_us": head["propose_us"],
        "commit_us": head["commit_us"],
        "setup_s": head["setup_s"],
        "copy_GBps": copy_gbs,
        "kernel_avg_us": head["kernel_avg_us"],
        "roofline": {k: droof[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")},
        "roofline_kernel": dom,
        "rooflines": head["rooflines"],
    }
    if "mixed" in res and head_prec != "mixed":
        m = summary("mixed")
        out["mixed"] = {"value": m["value"], "ms_per_step": m["ms_per_step"],
                        "host_driven_ms_per_step": m["host_driven_ms_per_step"],
                        "valid_proposals_per_s": m["valid_per_s"],
                        "propose_only_per_s": m["propose_only_per_s"], "propose_us": m["propose_us"],
                        "commit_us": m["commit_us"],
                        "dtype": "f32 fine-level evaluation, f64 difference/far field/commit",
                        "kernel_avg_us": m["kernel_avg_us"], "rooflines": m["rooflines"]}
    if res_exact:
        out["exact_self_image"] = {}
        for pr in precs:
            m = summary(pr, exact=True)
            out["exact_self_image"][pr] = {
                "value": m["value"], "ms_per_step": m["ms_per_step"], "host_driven_ms_per_step": m["host_driven_ms_per_step"],
                "propose_us": m["propose_us"], "commit_us": m["commit_us"], "setup_s": m["setup_s"],
                "kernel_avg_us": m["kernel_avg_us"], "rooflines": m["rooflines"],
                "note": "self_image=1: the moving charge's own copies by the exact Ewald change per hop instead of the "
                        "V_box sum + constant + 1/2 dE.R'dK (no per-charge hop table)"}
    if res_levels:
        out["per_level"] = {}
        for pr in precs:
            m = summary(pr, levels=True)
            out["per_level"][pr] = {
                "value": m["value"], "ms_per_step": m["ms_per_step"], "host_driven_ms_per_step": m["host_driven_ms_per_step"],
                "propose_us": m["propose_us"], "commit_us": m["commit_us"], "setup_s": m["setup_s"],
                "kernel_avg_us": m["kernel_avg_us"], "rooflines": m["rooflines"],
                "note": "per_level=1: local expansions kept per level; an accept updates the interaction-list cells "
                        "of each level (k_levels) instead of every fine cell (k_sweep); proposals add the coarser "
                        "levels per site (k_coarse_s2)"}
    if res_both:
        out["per_level_exact_self_image"] = {}
        for pr in precs:
            m = summary(pr, exact=True, levels=True)
            out["per_level_exact_self_image"][pr] = {
                "value": m["value"], "ms_per_step": m["ms_per_step"], "host_driven_ms_per_step": m["host_driven_ms_per_step"],
                "propose_us": m["propose_us"], "commit_us": m["commit_us"], "setup_s": m["setup_s"],
                "kernel_avg_us": m["kernel_avg_us"], "rooflines": m["rooflines"],
                "note": "per_level=1 and self_image=1 together"}
    if not args.skip_batch:
        out["batched"] = batched_summary(args)
        out["slab"] = run_slab(max(args.steps, 5), args.warmup, W.BASE_SEED + 6)
    if not args.skip_cpu:
        try:
            out["cpu_baseline"] = cpu_baseline(n, N, L, p, hops, seed)
        except Exception as e:  # the oracle is optional for the GPU figures
            out["cpu_baseline"] = {"error": str(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
