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
                  "sweep": "kernels_commit.hip", "b_site": "kernels_propose.hip", "b_slot": "kernels_propose.hip",
                  "b_sweep": "kernels_commit.hip"}


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


def accuracy_sample(sites, n, L, hops):
    """the bounded sample of the oracle leg: every valid hop of the charges in
    the 2x2x2 block of fine cells at the middle of the box; returns (charge
    index, target site, slot index i * K + k) of each slot"""
    from oracle import lattice_targets  # the oracle leg's own bookkeeping
    nc = 2 ** (L - 1)
    w = n / nc
    xyz = W.site_xyz(sites, n)
    cells = np.floor(xyz / w).astype(int)
    idx_c = np.nonzero(np.all((cells >= nc // 2) & (cells < nc // 2 + 2), axis=1))[0]
    t, valid = lattice_targets(sites, n, hops, True)  # occupancy of every charge
    t, valid = t[idx_c], valid[idx_c]
    K = len(hops)
    v = valid.reshape(-1)
    charge = np.repeat(idx_c, K)[v]
    slot = (np.repeat(idx_c, K) * K + np.tile(np.arange(K), len(idx_c)))[v]
    return charge, t.reshape(-1)[v], slot


def sample_slots(n, N, L, hops):
    """slot indices of the oracle leg's sample, computed without the oracle: the
    charges in the 2x2x2 block of fine cells at the middle of the box, every hop"""
    sites, xyz, q = W.lattice_charges(n, N, W.BASE_SEED + 4)
    nc = 2 ** (L - 1)
    cells = np.floor(xyz / (n / nc)).astype(int)
    idx_c = np.nonzero(np.all((cells >= nc // 2) & (cells < nc // 2 + 2), axis=1))[0]
    K = len(hops)
    return (idx_c[:, None] * K + np.arange(K)[None, :]).reshape(-1)


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
    # the first pass's dU of the oracle leg's sample (accuracy report)
    pick = torch.as_tensor(sample_slots(n, N, L, hops), device="cuda")
    sample_dU = dU.reshape(-1)[pick].cpu().numpy()
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
    # the kernels of the device-driven step, timed by HIP events as plain launches
    b.set_profiling(True)
    nprof = 5
    b.step(rng.random((nprof, 1)))
    graph_k = {}
    for name in ["b_site", "b_slot", "b_count", "b_select", "b_move_dU", "b_move_dU_side", "b_frow", "b_sweep",
                 "b_levels", "b_coarse_s2", "b_path", "b_book", "b_far_refresh", "b_cheb_a", "b_cheb_b", "b_finish"]:
        ms, k = b.kernel_time(name)
        if k:
            graph_k[name] = {"us_per_step": ms / nprof * 1e3, "launches_per_step": k / nprof}
    b.set_profiling(False)
    b.close()
    ctx.close()
    return dict(setup_s=setup_s, host_ms_per_step=1e3 * wall / steps, ms_per_step=1e3 * graph_wall / steps,
                propose_ms=1e3 * propose_wall / steps, commit_us=1e6 * commit_wall / steps, kernels=ktimes,
                valid_slots=valid, U0=U0, tuning=tuning, graph_kernels=graph_k, sample_dU=sample_dU)


def batch_contexts(precision, p=10, count=256, per_level=False, self_image="expansion"):
    """the replicas of the batched workload: N_r log-uniform in [1000, 65536],
    lattice side n_r = ceil((2 N_r)^(1/3)) (about 50 % occupancy), depth by the
    level rule, periodic, p = 10"""
    from paper_1905_04065_amd import Context
    Ns, ns, Ls = W.replica_sizes(count)
    ctxs = []
    for r in range(count):
        sites, xyz, q = W.replica_system(r, Ns[r], ns[r])
        c = Context(xyz, q, a=float(ns[r]), levels=int(Ls[r]), order=p, bc="periodic", precision=precision,
                    lattice_n=int(ns[r]), device=0, per_level=per_level, self_image=self_image)
        c.initialise()
        ctxs.append(c)
        if (r + 1) % 64 == 0:
            log(f"[batch] {precision}: {r + 1}/{count} replicas set up")
    return ctxs, Ns, ns


def run_batched(precision, steps, warmup, seed, tune=True, keep=False, per_level=False, self_image="expansion"):
    """config-5 steps of all replicas as one captured graph per step"""
    import torch

    from paper_1905_04065_amd import Batch
    t0 = time.perf_counter()
    ctxs, Ns, ns = batch_contexts(precision, per_level=per_level, self_image=self_image)
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
    nprof = 3
    b.step(rng.random((nprof, R)))
    phases = {}
    for name in ["b_coarse", "b_coarse_s2", "b_site", "b_slot", "b_count", "b_select", "b_move_dU", "b_move_dU_side",
                 "b_frow", "b_sweep", "b_levels", "b_path", "b_book", "b_far_refresh", "b_cheb_a", "b_cheb_b",
                 "b_finish"]:
        ms, n = b.kernel_time(name)
        if n:
            phases[name] = ms / nprof * 1e3  # per step (some phases are several launches)
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


def cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0))}


def guarded(d, ref, scale):
    e = np.abs(d - ref) / np.maximum(np.abs(ref), scale)
    return float(np.max(e)), float(np.mean(e))


def paper_rel(d, ref):
    """the per-proposal relative error of the paper's error study (Sec. 6.1): mean and max"""
    r = np.abs(d - ref) / np.abs(ref)
    return float(np.mean(r)), float(np.max(r))


def cpu_baseline(n, N, L, p, hops, seed, runs, budget_s=20.0):
    """The oracle leg.  Timing: O-fmm (FP64, OpenMP) on the host cores, on a
    bounded sample (every valid hop of the charges in the 2x2x2 block of fine
    cells at the middle of the box), after the cells those proposals touch have
    been formed; O-exact (tin-foil Ewald, FFT lattice form) on the same sample.
    Accuracy: the GPU's dU of the same sample slots (first proposal pass of each
    variant's context) against O-fmm of the same variant and against O-exact."""
    import oracle as O

    sites, xyz, q = W.lattice_charges(n, N, seed)
    charge, tsite, slot = accuracy_sample(sites, n, L, hops)
    pos = np.searchsorted(sample_slots(n, N, L, hops), slot)
    tgt = W.site_xyz(tsite, n)
    t0 = time.perf_counter()
    f = O.FmmKmc(xyz, q, float(n), L, p, "periodic", lazy=True)
    setup = time.perf_counter() - t0
    for x in np.concatenate([xyz[np.unique(charge)], tgt]):
        f.local(f.fine_cell_of(x))
    t0 = time.perf_counter()
    reps = 0
    while True:
        d_fmm = f.propose(charge, tgt)
        reps += 1
        el = time.perf_counter() - t0
        if el > budget_s / 4 or reps >= 50:
            break
    rate = reps * len(charge) / el
    f.close()
    t0 = time.perf_counter()
    E = O.LatticeEwald(sites, q, n)
    exact = E.dU_many(charge, tsite)
    t_exact = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", 0)) or len(os.sched_getaffinity(0))
    base = dict(value=rate, unit="proposals/s", cores=threads, kind="oracle",
                sample=f"{len(charge)} valid slots (all {len(hops)} hops of the charges in a 2x2x2 block of fine cells) "
                       f"x {reps} repetitions, FP64 O-fmm with OpenMP; octree upward pass ({setup:.1f} s) and "
                       f"formation of the touched cells' local expansions excluded",
                o_exact_proposals_per_s=len(charge) / t_exact,
                o_exact_note="tin-foil Ewald, FFT lattice form (one 3-D FFT of the site charges, then the "
                             "real-space sum per slot), single thread numpy; setup included", **cpu_info())
    # accuracy of every variant the GPU ran, on the same sample
    acc = {}
    scale = float(np.mean(np.abs(exact)))
    for variant, (self_image, per_level) in {"paper": ("expansion", False), "exact_self_image": ("exact", False),
                                             "per_level": ("expansion", True),
                                             "per_level_exact_self_image": ("exact", True)}.items():
        if variant not in runs:
            continue
        ref = d_fmm if variant == "paper" else None
        if ref is None:
            g = O.FmmKmc(xyz, q, float(n), L, p, "periodic", lazy=True, self_image=self_image, per_level=per_level)
            ref = g.propose(charge, tgt)
            g.close()
        o_mean, o_max = paper_rel(ref, exact)
        acc[variant] = {"o_fmm_vs_o_exact_mean_rel": o_mean, "o_fmm_vs_o_exact_max_rel": o_max}
        for pr, r in runs[variant].items():
            d = r["sample_dU"][pos]
            gmax, gmean = guarded(d, ref, scale)
            e_mean, e_max = paper_rel(d, exact)
            acc[variant][pr] = {"vs_o_fmm_guarded_max": gmax, "vs_o_fmm_guarded_mean": gmean,
                                "vs_o_fmm_guarded_max_floor_1e-3_mean": guarded(d, ref, 1e-3 * scale)[0],
                                "vs_o_exact_mean_rel": e_mean, "vs_o_exact_max_rel": e_max}
    acc["sample"] = f"{len(charge)} slots of the first proposal pass (initial configuration); guarded error floor " \
                    f"<|dU|> = {scale:.4f}"
    return base, acc


def accuracy_small_configs():
    """configs 1, 2, 3 and two replicas of config 5 against the oracles, as the GPU
    parity tests run them (oracle leg of the benchmark)"""
    import torch

    import oracle as O
    from paper_1905_04065_amd import Batch, Context
    out = {}

    def lattice_pass(ctx, hops):
        dU, mask = ctx.propose_lattice(hops)
        torch.cuda.synchronize()
        return dU.cpu().numpy().reshape(-1), mask.cpu().numpy().reshape(-1).astype(bool)

    # config 1: every slot vs O-fmm and vs the direct sum
    sites, xyz, q, c = W.config_system(1)
    hops = W.hops(c["hops"])
    ctx = Context(xyz, q, a=c["a"], levels=c["L"], order=c["p"], bc="free", lattice_n=c["n"], device=0)
    ctx.initialise()
    d, m = lattice_pass(ctx, hops)
    ctx.close()
    t, v = O.lattice_targets(sites, c["n"], hops, False)
    v = v.reshape(-1)
    idx = np.repeat(np.arange(len(q)), len(hops))[v]
    tgt = W.site_xyz(t.reshape(-1)[v], c["n"])
    ref = O.FmmKmc(xyz, q, c["a"], c["L"], c["p"], "free").propose(idx, tgt)
    ex = O.direct_dU(xyz, q, idx, tgt)
    sc = float(np.mean(np.abs(ref)))
    out["config1"] = {"slots": int(v.sum()), "vs_o_fmm_guarded_max": guarded(d[v], ref, sc)[0],
                      "vs_o_fmm_guarded_mean": guarded(d[v], ref, sc)[1],
                      "vs_o_exact_mean_rel": paper_rel(d[v], ex)[0], "vs_o_exact_max_rel": paper_rel(d[v], ex)[1]}
    # config 3: mixed, every slot before and after 10^4 accepted moves replayed by O-fmm; energy drift
    sites, xyz, q, c = W.config_system(3)
    ctx = Context(xyz, q, a=c["a"], levels=c["L"], order=c["p"], bc="free", precision="mixed", lattice_n=c["n"],
                  device=0)
    ctx.initialise()
    ref = O.FmmKmc(xyz, q, c["a"], c["L"], c["p"], "free")
    d0, _ = lattice_pass(ctx, hops)
    t, v = O.lattice_targets(sites, c["n"], hops, False)
    v = v.reshape(-1)
    idx = np.repeat(np.arange(len(q)), len(hops))
    r0 = ref.propose(idx[v], W.site_xyz(t.reshape(-1)[v], c["n"]))
    sc = float(np.mean(np.abs(r0)))
    ex0 = O.direct_dU(xyz, q, idx[v], W.site_xyz(t.reshape(-1)[v], c["n"]))
    u = W.commit_choices(c["commits"], W.BASE_SEED + 3)
    cur = sites.copy()
    worst = 0.0
    for s_ in range(c["commits"]):
        t, vv = O.lattice_targets(cur, c["n"], hops, False)
        vs = np.nonzero(vv.reshape(-1))[0]
        s = vs[int(u[s_] * len(vs))]
        i = int(s // len(hops))
        new = W.site_xyz([t.reshape(-1)[s]], c["n"])[0]
        dg, dr = ctx.accept(i, new), ref.accept(i, new)
        worst = max(worst, abs(dg - dr) / max(abs(dr), sc))
        cur[i] = t.reshape(-1)[s]
    d1, _ = lattice_pass(ctx, hops)
    t, v1 = O.lattice_targets(cur, c["n"], hops, False)
    v1 = v1.reshape(-1)
    r1 = ref.propose(idx[v1], W.site_xyz(t.reshape(-1)[v1], c["n"]))
    out["config3_mixed"] = {"vs_o_fmm_guarded_max_before": guarded(d0[v], r0, sc)[0],
                            "vs_o_exact_mean_rel_before": paper_rel(d0[v], ex0)[0],
                            "vs_o_fmm_guarded_max_after_1e4_commits": guarded(d1[v1], r1, sc)[0],
                            "accepted_dU_vs_o_fmm_max": worst,
                            "energy_drift_after_1e4_commits": abs(ctx.energy - ref.energy)}
    ctx.close()
    ref.close()
    # config 2: 100 steps with commit, then 512 sampled slots vs O-fmm and tin-foil Ewald
    sites, xyz, q, c = W.config_system(2)
    hops = W.hops(c["hops"])
    K = len(hops)
    ctx = Context(xyz, q, a=c["a"], levels=c["L"], order=c["p"], bc="periodic", lattice_n=c["n"], device=0)
    ctx.initialise()
    ref = O.FmmKmc(xyz, q, c["a"], c["L"], c["p"], "periodic", lazy=True)
    u = W.commit_choices(c["steps"], W.BASE_SEED + 2)
    cur = sites.copy()
    worst = 0.0
    for s_ in range(c["steps"]):
        d, m = lattice_pass(ctx, hops)
        t, vv = O.lattice_targets(cur, c["n"], hops, True)
        vs = np.nonzero(vv.reshape(-1))[0]
        s = vs[int(u[s_] * len(vs))]
        i = int(s // K)
        new = W.site_xyz([t.reshape(-1)[s]], c["n"])[0]
        dg, dr = ctx.accept(i, new), ref.accept(i, new)
        worst = max(worst, abs(dg - dr) / max(abs(dr), 0.05))
        cur[i] = t.reshape(-1)[s]
    d, m = lattice_pass(ctx, hops)
    t, vv = O.lattice_targets(cur, c["n"], hops, True)
    vv = vv.reshape(-1)
    pick = np.random.default_rng(W.BASE_SEED + 20).choice(np.nonzero(vv)[0], 512, replace=False)
    dr = ref.propose(pick // K, W.site_xyz(t.reshape(-1)[pick], c["n"]))
    ex = O.LatticeEwald(cur, q, c["n"]).dU_many(pick // K, t.reshape(-1)[pick])
    sc = float(np.mean(np.abs(d[vv])))
    out["config2"] = {"accepted_dU_vs_o_fmm_max_100_steps": worst,
                      "vs_o_fmm_guarded_max_512_sampled_after": guarded(d[pick], dr, sc)[0],
                      "vs_o_exact_mean_rel_512_sampled": paper_rel(d[pick], ex)[0],
                      "vs_o_exact_max_rel_512_sampled": paper_rel(d[pick], ex)[1]}
    ctx.close()
    ref.close()
    # config 5: the largest and the smallest replica (p = 10, mixed, batched), 256 sampled slots each
    Ns, ns, Ls = W.replica_sizes()
    res5 = {}
    for r in (int(np.argmax(Ns)), int(np.argmin(Ns))):
        sites, xyz, q = W.replica_system(r, Ns[r], ns[r])
        n = int(ns[r])
        ctx = Context(xyz, q, a=float(n), levels=int(Ls[r]), order=10, bc="periodic", precision="mixed",
                      lattice_n=n, device=0)
        ctx.initialise()
        b = Batch([ctx], W.HOPS6)
        mv, st, _ = (x.cpu().numpy() for x in b.step(np.full((1, 1), 0.37)))
        dnow, mnow = lattice_pass(ctx, W.HOPS6)
        b.close()
        cur = np.floor(ctx.positions().cpu().numpy()).astype(np.int64) @ np.array([n * n, n, 1])
        ctx.close()
        t, vv = O.lattice_targets(cur, n, W.HOPS6, True)
        vv = vv.reshape(-1)
        pick = np.random.default_rng(W.BASE_SEED + 70 + r).choice(np.nonzero(vv)[0], 256, replace=False)
        ref = O.FmmKmc(xyz, q, float(n), int(Ls[r]), 10, "periodic", lazy=True)
        ref.accept(int(mv[0, 0]), W.site_xyz([int(st[0, 0])], n)[0])  # the same move, replayed
        dr = ref.propose(pick // 6, W.site_xyz(t.reshape(-1)[pick], n))
        ref.close()
        ex = O.LatticeEwald(cur, q, n).dU_many(pick // 6, t.reshape(-1)[pick])
        sc = float(np.mean(np.abs(dnow[vv])))
        res5[f"replica{r}_n{n}_N{int(Ns[r])}_L{int(Ls[r])}"] = {
            "vs_o_fmm_guarded_max_256_sampled": guarded(dnow[pick], dr, sc)[0],
            "vs_o_exact_mean_rel_256_sampled": paper_rel(dnow[pick], ex)[0]}
    out["config5_mixed_after_one_batched_step"] = res5
    return out


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


def batched_rooflines(run, precision, p=10, count=256):
    """work of the batched step's site and sweep phases over all replicas:
    the site phase against HBM (algorithmic bytes: the fine-level expansions
    once, the site tables, the potentials out) with the near-field box entries
    per second beside it (the general-lattice bodies are bound by LDS and
    VALU, not HBM); the sweep against FP64 peak"""
    Ns, ns, Ls = W.replica_sizes(count)
    nt = (p + 1) ** 2
    mixed = precision == "mixed"
    nbytes = flop = entries = 0
    for N, n, L in zip(Ns, ns, Ls):
        N, n, L = int(N), int(n), int(L)
        nc = 2 ** (L - 1)
        M = nc ** 3
        sites = n ** 3
        nbytes += M * nt * (4 if mixed else 8) + (M * 8 if mixed else 0) + sites * ((4 if mixed else 8) + 4 + 8) \
            + N * 8 + n * n * (p + 1) * 8
        flop += M * 54 * P2L_FLOP * nt / 169.0
        # near-field box entries: per axis the planes of the three cells around each site's cell
        w = n / nc
        cell = np.minimum(np.floor((np.arange(n) + 0.5) / w).astype(int), nc - 1)
        per = np.bincount(cell, minlength=nc)
        ext = per[(cell - 1) % nc] + per[cell] + per[(cell + 1) % nc]
        entries += int(ext.sum()) ** 3
    ph = run["phase_us"]
    out = {}
    if "b_site" in ph:
        us = ph["b_site"]
        ach = nbytes / (us * 1e-6) / 1e9
        out["b_site"] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ach / HBM_PEAK_GBS, "algorithmic_bytes": nbytes, "avg_us": us,
                         "near_field_box_entries": entries, "box_entries_per_s": entries / (us * 1e-6),
                         "note": "all three site launches per step (2x2x2 body; the general lattices' local "
                                 "expansion pass and near-field pass); the near field is LDS- and VALU-bound"}
    if "b_sweep" in ph:
        us = ph["b_sweep"]
        ach = flop / (us * 1e-6) / 1e12
        out["b_sweep"] = {"bound": "alu", "achieved": ach, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                          "frac": ach / FP64_PEAK_TFLOPS, "algorithmic_flop": flop, "avg_us": us}
    return out


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
    log("[batch] mixed, exact self-image term")
    mixed_exact = run_batched("mixed", steps, args.warmup, seed, self_image="exact")
    log("[batch] mixed, per-level expansions and exact self-image term")
    mixed_levels = run_batched("mixed", steps, args.warmup, seed, per_level=True, self_image="exact")
    slots = mixed["slots_per_step"]
    rooflines = {pr: batched_rooflines(r, pr) for pr, r in (("mixed", mixed), ("fp64", fp64))}
    return {
        "rooflines": rooflines,
        "workload": f"{mixed['replicas']} periodic replicas, N_r log-uniform in [1000, 65536] (sum {slots // 6}), "
                    "50 % lattice occupancy, 6 hops, p=10, one accepted move per replica per step",
        "slots_per_step": slots,
        "mixed_batched": {"proposals_per_s": slots / (mixed["ms_per_step"] / 1e3), **mixed},
        "fp64_batched": {"proposals_per_s": slots / (fp64["ms_per_step"] / 1e3), **fp64},
        "fp64_host_driven_one_replica_at_a_time": {
            "proposals_per_s": slots / (plain["ms_per_step"] / 1e3), **plain,
            "note": "each replica through the single-context API with the selection on the host (one host "
                    "synchronisation per replica): mostly host overhead, not a kernel comparison"},
        "speedup_mixed_batched_vs_fp64_batched": fp64["ms_per_step"] / mixed["ms_per_step"],
        "mixed_batched_exact_self_image": {"proposals_per_s": slots / (mixed_exact["ms_per_step"] / 1e3),
                                           **mixed_exact},
        "mixed_batched_per_level_exact_self_image": {"proposals_per_s": slots / (mixed_levels["ms_per_step"] / 1e3),
                                                     **mixed_levels},
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
    ap.add_argument("--variants", default="exact,per_level,both",
                    help="variants run beside the paper's terms: comma list of exact (exact self-image term), "
                         "per_level (per-level expansions), both")
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
    want = set(v.strip() for v in args.variants.split(",") if v.strip())
    if args.skip_exact_self:
        want -= {"exact", "both"}
    if args.skip_per_level:
        want -= {"per_level", "both"}
    res_exact = {} if "exact" not in want else {
        pr: run_gpu(pr, n, N, L, p, hops, args.steps, args.warmup, seed, self_image="exact") for pr in precs}
    res_levels = {} if "per_level" not in want else {
        pr: run_gpu(pr, n, N, L, p, hops, args.steps, args.warmup, seed, per_level=True) for pr in precs}
    res_both = {} if "both" not in want else {
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

    def graph_rooflines(r, pr, exact, counters=False):
        """rooflines of the kernels the device-driven step runs (HIP events around
        plain launches of the batched kernels, one launch each per step);
        counters: take HBM traffic from the committed rocprofv3 counters"""
        gk = r["graph_kernels"]
        traffic = profiled_traffic(tag, pr) if counters else {}
        out_ = {}
        for name, kern in (("b_site", "site_phi_s2"), ("b_slot", "slot_lattice"), ("b_sweep", "sweep")):
            if name not in gk:
                continue
            us = gk[name]["us_per_step"]
            bound, amount, unit = kernel_work(kern, n, N, K, p, pr, exact)
            if bound == "hbm":
                ach = amount / (us * 1e-6) / 1e9
                out_[name] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": ach / HBM_PEAK_GBS, "frac_of_copy": ach / copy_gbs, "avg_us": us,
                              "algorithmic_bytes": amount, "traffic": traffic.get(name)}
            else:
                ach = amount / (us * 1e-6) / 1e12
                out_[name] = {"bound": "alu", "achieved": ach, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                              "frac": ach / FP64_PEAK_TFLOPS, "avg_us": us, "algorithmic_flop": amount,
                              "hbm_bytes": sweep_bytes(n, p, pr), "traffic": traffic.get(name)}
        if "b_site" in out_ and "b_slot" in out_:
            tb = out_["b_site"]["algorithmic_bytes"] + out_["b_slot"]["algorithmic_bytes"]
            tus = out_["b_site"]["avg_us"] + out_["b_slot"]["avg_us"]
            # the survey's count of the proposal pass (S0-S3): 640 MB FP64, 460 MB mixed at this size
            sb = (640e6 if pr == "fp64" else 460e6) * (N * K) / 26e6
            out_["proposal_pass"] = {"bound": "hbm", "algorithmic_bytes": tb, "avg_us": tus,
                                     "achieved": tb / (tus * 1e-6) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                     "frac": tb / (tus * 1e-6) / 1e9 / HBM_PEAK_GBS,
                                     "frac_with_survey_bytes": sb / (tus * 1e-6) / 1e9 / HBM_PEAK_GBS}
        return out_

    head = summary(head_prec)
    groof = graph_rooflines(res[head_prec], head_prec, False, counters=True)
    # the kernel of the headline (device-driven) step with the largest time per step
    gdom = max((k for k in ("b_site", "b_slot", "b_sweep") if k in groof), key=lambda k: groof[k]["avg_us"])
    droof = dict(groof[gdom])
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
                               f"L={L}, p={p}, one accepted move per step; the paper's terms (fine-level sweep "
                               "at each accept, Sec. 3.1 self terms)",
                   "global_batch": slots, "parallelism": "single GPU"},
        "valid_proposals_per_s": head["valid_per_s"],
        "valid_slots": res[head_prec]["valid_slots"],
        "propose_only_per_s": head["propose_only_per_s"],
        "propose_us": head["propose_us"],
        "commit_us": head["commit_us"],
        "setup_s": head["setup_s"],
        "copy_GBps": copy_gbs,
        "roofline": {k: droof[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")},
        "roofline_kernel": gdom,
        "graph_step_rooflines": groof,
        "graph_step_kernel_us": res[head_prec]["graph_kernels"],
        "host_driven_kernel_avg_us": head["kernel_avg_us"],
        "host_driven_rooflines": head["rooflines"],
    }
    if "mixed" in res and head_prec != "mixed":
        m = summary("mixed")
        out["mixed"] = {"value": m["value"], "ms_per_step": m["ms_per_step"],
                        "host_driven_ms_per_step": m["host_driven_ms_per_step"],
                        "valid_proposals_per_s": m["valid_per_s"],
                        "propose_only_per_s": m["propose_only_per_s"], "propose_us": m["propose_us"],
                        "commit_us": m["commit_us"],
                        "dtype": "f32 fine-level evaluation, f64 difference/far field/commit",
                        "speedup_vs_fp64": head["ms_per_step"] / m["ms_per_step"],
                        "graph_step_rooflines": graph_rooflines(res["mixed"], "mixed", False, counters=True),
                        "graph_step_kernel_us": res["mixed"]["graph_kernels"],
                        "host_driven_kernel_avg_us": m["kernel_avg_us"]}
    notes = {"exact_self_image": "self_image=1: the moving charge's own copies by the exact Ewald change per hop "
                                 "instead of the V_box sum + constant + 1/2 dE.R'dK (no per-charge hop table)",
             "per_level": "per_level=1: local expansions kept per level; an accept updates the interaction-list cells "
                          "of each level (k_levels) instead of every fine cell (k_sweep); proposals add the coarser "
                          "levels per site (k_coarse_s2)",
             "per_level_exact_self_image": "per_level=1 and self_image=1 together"}
    runs = {"paper": res}
    variants = {}
    for key, rr, exact, levels in (("exact_self_image", res_exact, True, False), ("per_level", res_levels, False, True),
                                   ("per_level_exact_self_image", res_both, True, True)):
        if not rr:
            continue
        runs[key] = rr
        variants[key] = {"note": notes[key]}
        for pr in precs:
            m = summary(pr, exact=exact, levels=levels)
            variants[key][pr] = {"value": m["value"], "ms_per_step": m["ms_per_step"],
                                 "speedup_vs_paper_fp64": head["ms_per_step"] / m["ms_per_step"],
                                 "host_driven_ms_per_step": m["host_driven_ms_per_step"],
                                 "propose_us": m["propose_us"], "commit_us": m["commit_us"], "setup_s": m["setup_s"],
                                 "graph_step_kernel_us": rr[pr]["graph_kernels"],
                                 "graph_step_rooflines": graph_rooflines(rr[pr], pr, exact),
                                 "host_driven_kernel_avg_us": m["kernel_avg_us"]}
    if variants:
        out["variants"] = variants
        best = min(((k, pr) for k in variants for pr in precs), key=lambda kp: variants[kp[0]][kp[1]]["ms_per_step"])
        out["best_variant"] = {"variant": best[0], "precision": best[1],
                               "value": variants[best[0]][best[1]]["value"],
                               "ms_per_step": variants[best[0]][best[1]]["ms_per_step"],
                               "speedup_vs_paper_fp64": variants[best[0]][best[1]]["speedup_vs_paper_fp64"]}
    if not args.skip_batch:
        out["batched"] = batched_summary(args)
        out["slab"] = run_slab(max(args.steps, 5), args.warmup, W.BASE_SEED + 6)
    if not args.skip_cpu:
        try:
            out["cpu_baseline"], acc = cpu_baseline(n, N, L, p, hops, seed, runs)
            out["accuracy"] = {"config4_sample": acc}
            if not args.quick:
                out["accuracy"].update(accuracy_small_configs())
        except Exception as e:  # the oracle is optional for the GPU figures
            out["cpu_baseline"] = {"error": str(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
