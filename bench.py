"""Benchmark: dU proposals/s and accepted-move commit time of FMM-KMC on one MI355X.

Workload: periodic cubic box, 128^3 site lattice (spacing 1), N = 10^6 neutral
+-1 charges on seeded random sites, 26 hop targets per charge (first, second
and third neighbour shells: 26M proposal slots per step), octree depth L = 7,
expansion order p = 12; FP64 and mixed precision.

A step is one pass of the whole hot path: the energy change of every slot
(propose) and one accepted move (commit: dU recomputed, every fine-level local
expansion, the multipole path on every level and the far field updated).  The
accepted move is a seeded uniform choice among the valid slots that does not
look at dU.  Inputs are resident on the GPU before timing starts; the one-time
setup (octree build) is timed separately and not part of a step.

Prints one JSON line.  Options: --steps K --warmup W --gpus 1 [--skip-cpu]
[--precision fp64|mixed|both] [--quick] (a small periodic system for a smoke run).
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

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
FP64_PEAK_TFLOPS = 78.6


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_bytes(kernel, n, N, K, p, precision):
    """Bytes one launch must move at minimum (each input read once, each output written once)."""
    nt = (p + 1) ** 2
    sites = n ** 3
    cells = sites // 8
    if kernel == "site_phi_s2":
        psi = cells * nt * (8 if precision == "fp64" else 4) + (0 if precision == "fp64" else cells * 8)
        charges = sites * (8 if precision == "fp64" else 4)
        far = n * n * (p + 1) * 8 + n * (p + 1) * 8
        return psi + charges + far + sites * 8
    if kernel == "slot_lattice":
        per_slot = 8 + 1 + 8          # dU out, mask out, F in
        per_charge = 4 + 8            # site, q
        return N * K * per_slot + N * per_charge + sites * 8 + sites * 4  # phi per site, site occupancy
    if kernel == "sweep":
        return 2 * cells * nt * 8 + (cells * nt * 4 if precision == "mixed" else 0)
    raise KeyError(kernel)


def run_gpu(precision, n, N, L, p, hops, steps, warmup, seed):
    import torch

    from paper_1905_04065_amd import Context

    sites, xyz, q = W.lattice_charges(n, N, seed)
    K = len(hops)
    log(f"[{precision}] create n={n} N={N} L={L} p={p} K={K}")
    t0 = time.perf_counter()
    ctx = Context(xyz, q, a=float(n), levels=L, order=p, bc="periodic", precision=precision, lattice_n=n,
                  device=0)
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
    names = ["site_phi_s2", "site_phi", "slot_lattice", "sweep", "path", "far_refresh", "cheb_a", "cheb_b", "f_rows",
             "f_row1", "book", "move_dU"]
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
    ctx.close()
    return dict(setup_s=setup_s, ms_per_step=1e3 * wall / steps, propose_ms=1e3 * propose_wall / steps,
                commit_us=1e6 * commit_wall / steps, kernels=ktimes, valid_slots=valid, U0=U0)


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
    t, valid = W.lattice_targets(sites[idx_c], n, hops, True)
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="both", choices=["fp64", "mixed", "both"])
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--quick", action="store_true", help="small periodic system (64^3, N=1e5, L=6)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU decomposition is "
              "described in DESIGN.md but not built", file=sys.stderr)
        sys.exit(2)
    if args.quick:
        n, N, L, p, hops = 64, 100000, 6, 12, W.HOPS26
    else:
        n, N, L, p, hops = 128, 1000000, 7, 12, W.HOPS26
    seed = W.BASE_SEED + 4
    K = len(hops)
    precs = ["fp64", "mixed"] if args.precision == "both" else [args.precision]
    res = {pr: run_gpu(pr, n, N, L, p, hops, args.steps, args.warmup, seed) for pr in precs}
    head = res["fp64"] if "fp64" in res else res[precs[0]]
    slots = N * K
    step_ms = head["ms_per_step"]
    # dominant kernel of the propose pass and its roofline
    kt = head["kernels"]
    dom = max(["site_phi_s2", "slot_lattice"], key=lambda k: kt[k][0])
    ms, launches = kt[dom]
    avg_s = ms / max(launches, 1) / 1e3
    hprec = "fp64" if "fp64" in res else precs[0]
    bytes_ = algorithmic_bytes(dom, n, N, K, p, hprec)
    achieved = bytes_ / avg_s / 1e9
    out = {
        "metric": "dU proposals/sec at N=1e6, p=12 (FP64 vs mixed); accepted-move commit us",
        "value": slots / (step_ms / 1e3),
        "unit": "proposals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if hprec == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"periodic {n}^3 lattice, N={N} +-1 charges, {K} hops/charge ({slots} slots/step), "
                               f"L={L}, p={p}, one accepted move per step",
                   "global_batch": slots, "parallelism": "single GPU"},
        "propose_only_per_s": slots / (head["propose_ms"] / 1e3),
        "commit_us": head["commit_us"],
        "valid_slots": head["valid_slots"],
        "setup_s": head["setup_s"],
        "kernel_avg_us": {k: (v[0] / max(v[1], 1) * 1e3) for k, v in kt.items() if v[1] > 0},
        "roofline": {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "algorithmic_bytes": bytes_},
    }
    if "mixed" in res and "fp64" in res:
        m = res["mixed"]
        out["mixed"] = {"value": slots / (m["ms_per_step"] / 1e3), "ms_per_step": m["ms_per_step"],
                        "propose_only_per_s": slots / (m["propose_ms"] / 1e3), "commit_us": m["commit_us"],
                        "dtype": "f32 fine-level evaluation, f64 difference/far field/commit",
                        "kernel_avg_us": {k: (v[0] / max(v[1], 1) * 1e3) for k, v in m["kernels"].items()
                                          if v[1] > 0}}
        mk = m["kernels"][dom]
        mavg = mk[0] / max(mk[1], 1) / 1e3
        mb = algorithmic_bytes(dom, n, N, K, p, "mixed")
        out["mixed"]["roofline"] = {"kernel": dom, "achieved": mb / mavg / 1e9, "peak": HBM_PEAK_GBS,
                                    "frac": mb / mavg / 1e9 / HBM_PEAK_GBS}
    if not args.skip_cpu:
        try:
            out["cpu_baseline"] = cpu_baseline(n, N, L, p, hops, seed)
        except Exception as e:  # the oracle is optional for the GPU figures
            out["cpu_baseline"] = {"error": str(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
