"""Benchmark of the PQMC field-update sweep on one MI355X.

One step = one full sweep (forward l = 1..M, backward l = M..1) of the
whole hot path -- B-matrix propagation, field updates, Metropolis
decisions, QR stabilisation and inverse -- on the 40x40 Hubbard workload
(N = 1600, N_sigma = 800 per spin, U/t = 4, dtau = 0.05, M = 400,
k_tau = 10, seeded 1e-3 bond perturbation), FP64, inputs resident in HBM.

value = field updates per second of the headline scheme (2 M N single-site
field visits per sweep / wall time per sweep).  The other schemes are
reported beside it, with the update-only rate (the paper's metric: update
phase only) from HIP events on the library's stream.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "field-updates/s delayed & block-FB vs local, 40x40 Hubbard FP64; jobs/s+p99"
MI355X_FP64_PEAK_TFLOPS = 78.6
MI355X_HBM_TBPS = 8.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_chain(p, scheme, k=1, b=1, timing=True, fp32=False):
    """One walker run alone: one 64 x 64 tile of T per workgroup of the flush
    kernel (tile_chunks = 64), so that a single chain still fills the GPU."""
    from paper_2506_09611_amd import Chain, Scheme
    sc = {"local": Scheme.LOCAL, "delayed": Scheme.DELAYED, "block": Scheme.BLOCK_FB,
          "local_g": Scheme.LOCAL_G}[scheme]
    return Chain(p.hopping, p.trial_up, p.trial_dn, p.U, p.dtau, p.n_slices, p.stab_every,
                 p.seed, p.walker_id, scheme=sc, k=k, b=b, timing=timing, fp32=fp32,
                 tile_chunks=64)


def sparse_propagation(p):
    """(J, nnz) when the library propagates this problem with the Taylor
    series of the sparse H0 (at most 8 nonzeros per row, N <= 4096,
    ||dtau H0||_1 <= 1; J: the degree whose first dropped term is below
    2^-60), else None."""
    import numpy as np
    H = p.hopping
    w = int(max(np.count_nonzero(H[i]) for i in range(H.shape[0])))
    norm1 = p.dtau * float(np.max(np.sum(np.abs(H), axis=0)))
    if w > 8 or H.shape[0] > 4096 or norm1 > 1.0:
        return None
    J, term = 0, 1.0
    while norm1 > 0.0 and term * norm1 / (J + 1) > 2.0 ** -60:
        J += 1
        term *= norm1 / J
    return J, int(np.count_nonzero(H))


def kernel_work(p, cls, scheme, k, b, acc):
    """Algorithmic work of one launch of a kernel class: (flops, bytes, bound).
    Two spin sectors; Ns = N_sigma; T is Ns x Ns; U_R, U_L^T are N x Ns."""
    N, Ns = p.n_sites, p.n_up
    kk = k if scheme == "delayed" else b
    n_a = acc * kk
    if cls == "propagate":     # U_R and U_L^T: 2 spins x 2 products by e^{-+dtau H0}
        sp = sparse_propagation(p)
        if sp is not None:     # Taylor series of the sparse H0: read X, write Y once
            J, nnz = sp
            return 2 * 2 * 2.0 * J * nnz * Ns, 2 * 2 * 2 * N * Ns * 8.0, "hbm"
        return 8.0 * N * N * Ns, 2 * 2 * (N * N + 2 * N * Ns) * 8.0, "mfma"
    if cls == "tile":          # flush T -= Q P2_A (rank n_A) + panels U_g T, T L_g
        return 2 * (2.0 * Ns * Ns * n_a + 4.0 * Ns * Ns * kk), 2 * 2 * Ns * Ns * 8.0, "mfma"
    nt = -(-Ns // 64)
    if cls == "reduce":        # sum the W0 partials (ceil(Ns/64) strips x 2 chunks), two spins
        return 2.0 * 2 * nt * kk * kk, 2 * (2 * nt + 1) * kk * kk * 8.0, "hbm"
    if cls == "decide":        # kk x kk pivot sweeps, and the P2 (nt) and P1 (2) partial sums
        return (2 * 2.0 * n_a * kk * kk + 2 * (nt + 2) * kk * Ns,
                2 * ((nt + 2) * kk * Ns + 2 * kk * Ns + kk * kk) * 8.0, "alu")
    if cls == "local" and scheme == "local_g":   # read G, rank-1 write when accepted
        return 2 * 2.0 * acc * N * N, 2 * (1.0 + acc) * N * N * 8.0, "hbm"
    if cls == "local":         # read T (partials of y, Tv), rank-1 write when accepted
        return 2 * (2.0 + 4.0 * acc) * Ns * Ns, 2 * (1.0 + acc) * Ns * Ns * 8.0, "hbm"
    raise KeyError(cls)


def roofline(p, scheme, k, b, acc, ktimes, cls=None, walkers=1):
    """Roofline of one kernel class (default: the one with the largest device
    time), from its average launch duration on the library's stream; one
    launch covers `walkers` walkers."""
    live = {c: v for c, v in ktimes.items() if v[1] > 0}
    if not live or (cls is not None and cls not in live):
        return None
    if cls is None:
        cls = max(live, key=lambda c: live[c][0])
    tot, cnt = live[cls]
    avg = tot / cnt
    flops, nbytes, bound = kernel_work(p, cls, scheme, k, b, acc)
    flops, nbytes = flops * walkers, nbytes * walkers
    if bound == "hbm":
        achieved, peak, unit = nbytes / avg / 1e9, MI355X_HBM_TBPS * 1e3, "GB/s"
    else:
        achieved, peak, unit = flops / avg / 1e12, MI355X_FP64_PEAK_TFLOPS, "TFLOP/s"
    shares = {c: v[0] for c, v in ktimes.items() if v[1] > 0}
    total = sum(shares.values())
    return {"kernel": cls, "bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "traffic": None, "avg_launch_us": avg * 1e6,
            "launches": cnt, "flops_per_launch": flops, "bytes_per_launch": nbytes,
            "device_time_share": {c: v / total for c, v in shares.items()}}


TRAFFIC_FILES = {
    "tile": os.path.join(ROOT, "profiles", "tile_kernel_40x40_w8_delayed_k32_traffic.txt"),
    "local": os.path.join(ROOT, "profiles", "local_site_kernel_40x40_w8_traffic.txt"),
}


def measured_traffic(cls, scheme, k, walkers, workload, tile_chunks=None):
    """HBM bytes per launch of the tile kernel or the per-site local kernel
    from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE runs (scaled by the
    same counters on a plain copy of known size), or None when they do not
    cover this launch or the kernel source has changed since they were taken."""
    import hashlib
    path = TRAFFIC_FILES.get(cls)
    if path is None or not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            key, val = line.split(":", 1)
            rec[key.strip()] = val.strip()
    src = os.path.join(ROOT, "paper_2506_09611_amd", "csrc", "update.hip")
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if (rec.get("source_sha256") != digest or rec.get("scheme") != scheme
            or ("k" in rec and int(rec["k"]) != k) or int(rec.get("walkers", -1)) != walkers
            or rec.get("workload") != workload
            or ("tile_chunks" in rec and tile_chunks is not None
                and int(rec["tile_chunks"]) != tile_chunks)):
        return None
    return float(rec["traffic_bytes_per_launch"])


def make_walkers(p, scheme, k, b, W, streams, fp32=False, tile_chunks=0):
    """W walkers (walker_id 0..W-1) on each of the given streams (walker ids
    continue across streams): one lockstep batch per stream."""
    import dataclasses
    from paper_2506_09611_amd import Chain, Scheme
    sc = {"local": Scheme.LOCAL, "local_g": Scheme.LOCAL_G, "delayed": Scheme.DELAYED,
          "block": Scheme.BLOCK_FB}[scheme]
    out = []
    for si, st in enumerate(streams):
        for w in range(W):
            q = dataclasses.replace(p, walker_id=si * W + w)
            out.append(Chain(q.hopping, q.trial_up, q.trial_dn, q.U, q.dtau, q.n_slices,
                             q.stab_every, q.seed, q.walker_id, scheme=sc, k=k, b=b,
                             timing=True, fp32=fp32, stream=st, tile_chunks=tile_chunks))
    return out


def time_sweeps(chains, steps, warmup):
    """Wall time of `steps` sweeps of all chains (one lockstep batch per
    stream, the batches concurrent: pqmc_multi_sweep) and the statistics
    summed over chains and steps (phase times: the first batch's)."""
    import torch
    from paper_2506_09611_amd import multi_sweep
    for _ in range(warmup):
        multi_sweep(chains, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = [multi_sweep(chains, 1) for _ in range(steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    agg = {k: sum(s[0][k] for s in st) for k in st[0][0]}
    for k in ("proposed", "accepted", "flips", "low_margin", "negative", "field_updates"):
        agg[k] = sum(w[k] for s in st for w in s)
    agg["max_stab_drift"] = max(w["max_stab_drift"] for s in st for w in s)
    return t1 - t0, agg


def host_description():
    """CPU model, logical cores and the BLAS the oracle's NumPy calls."""
    import numpy as np
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    blas = {}
    try:
        dep = np.show_config(mode="dicts").get("Build Dependencies", {}).get("blas", {})
        blas = {"name": dep.get("name"), "version": dep.get("version")}
    except Exception:  # pragma: no cover
        pass
    try:
        from threadpoolctl import threadpool_info
        info = [i for i in threadpool_info() if i.get("user_api") == "blas"]
        if info:
            blas.update({"internal_api": info[0].get("internal_api"),
                         "threads": info[0].get("num_threads"),
                         "architecture": info[0].get("architecture")})
    except Exception:  # pragma: no cover
        pass
    return {"cpu_model": model, "logical_cores": os.cpu_count(), "blas": blas}


def _oracle_forward(q, scheme, k, b, visits):
    """Seconds per forward slice visit (propagation + update, with the
    stabilisations that fall inside) of the oracle walker, after its set-up."""
    import numpy as np
    from oracle.pqmc import Walker
    w = Walker(q, scheme, k=k, b=b)
    t0 = time.perf_counter()
    for l in range(1, visits + 1):
        w.prop_forward(l)
        w.update_slice(l, 0)
        if l % w.kt == 0:
            for s in range(2):
                w.UR[s] = np.linalg.qr(w.UR[s])[0]
                w.UL[s] = w.Lstack[s][l // w.kt].copy()
            w.refresh_T()
    return (time.perf_counter() - t0) / visits


def cpu_baseline(p, scheme, k, b, visits=20, one_core_visits=4):
    """The oracle timed on the host cores:
      * the 40x40 workload: `visits` forward slice visits of the headline
        scheme (two stabilisations at k_tau = 10) on all cores, and
        `one_core_visits` on one BLAS thread; a sweep is 2 M = 800 visits, so
        the per-visit rate is the sweep rate and s/sweep is extrapolated x 40;
      * 4x4 (c1) whole sweeps of the local, delayed (k = 16) and block (b = 8)
        updates, and one whole 16x16 (c2) sweep of the delayed update (k = 16),
        all cores.
    The projection of the 40x40 sample is shortened to M = 20 (the cost of a
    slice visit does not depend on M; the set-up of M = 400 would take
    minutes)."""
    import synth
    from oracle.pqmc import Walker
    host = host_description()
    try:
        from threadpoolctl import threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_limits = None
    threads = host["blas"].get("threads") or os.cpu_count()
    q = synth.workload("c3", n_slices=20, stab_every=10)
    sv = _oracle_forward(q, scheme, k, b, visits)
    rate = q.n_sites / sv
    one = None
    if threadpool_limits is not None:
        with threadpool_limits(limits=1, user_api="blas"):
            sv1 = _oracle_forward(q, scheme, k, b, one_core_visits)
        one = {"value": q.n_sites / sv1, "cores": 1, "s_per_slice_visit": sv1,
               "extrapolated_s_per_sweep": sv1 * 800, "visits": one_core_visits}
    whole = {}
    for name, wl, sch, kk, bb in [("c1 local", "c1", "local", 1, 1),
                                  ("c1 delayed k=16", "c1", "delayed", 16, 1),
                                  ("c1 block b=8", "c1", "block", 1, 8),
                                  ("c2 delayed k=16", "c2", "delayed", 16, 1)]:
        qq = synth.workload(wl)
        w = Walker(qq, sch, k=kk, b=bb)
        t0 = time.perf_counter()
        w.sweep()
        dt = time.perf_counter() - t0
        whole[name] = {"s_per_sweep": dt,
                       "field_updates_per_s": 2 * qq.n_slices * qq.n_sites / dt,
                       "acceptance": w.n_accepted / max(1, w.n_proposed)}
    c1l = whole["c1 local"]["s_per_sweep"]
    for name in ("c1 delayed k=16", "c1 block b=8"):
        whole[name]["speedup_vs_local"] = c1l / whole[name]["s_per_sweep"]
    return {"value": rate, "unit": "field-updates/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{scheme} k={k} b={b}: {visits} forward slice visits (propagation, "
                      f"update, two stabilisations) of the 40x40 lattice, N_sigma=800, "
                      f"projection shortened to M=20; per-visit rate = sweep rate "
                      f"({sv * 800:.0f} s per 800-visit sweep, extrapolated x40)",
            "s_per_slice_visit": sv, "extrapolated_s_per_sweep": sv * 800,
            "one_core": one, "whole_sweeps_all_cores": whole, "host": host}


def scheme_table(p, spec, window):
    """One walker, forward windows of `window` slice visits (propagation,
    updates, the stabilisations inside the window), for each delay rank and
    block size in spec ('delayed:8,16;block:1,4'), beside the local update."""
    import torch
    N = p.n_sites
    rows = []
    entries = [("local", 1)]
    for part in spec.split(";"):
        name, vals = part.split(":")
        entries += [(name, int(v)) for v in vals.split(",") if v]
    base = None
    for name, kb in entries:
        c = make_chain(p, name, k=kb if name == "delayed" else 1, b=kb if name == "block" else 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = c.forward_window(window)
        torch.cuda.synchronize()
        w = time.perf_counter() - t0
        row = {"scheme": name, "rank": kb, "field_updates_per_s": window * N / w,
               "update_only": window * N / st["t_update_s"] if st["t_update_s"] > 0 else None,
               "acceptance": st["accepted"] / max(1, st["proposed"])}
        if name == "local":
            base = row
        row["speedup_vs_local"] = row["field_updates_per_s"] / base["field_updates_per_s"]
        row["update_speedup_vs_local"] = (row["update_only"] / base["update_only"]
                                          if row["update_only"] and base["update_only"] else None)
        rows.append(row)
        log("table", row)
        c.close()
        del c
        torch.cuda.empty_cache()
    return {"walkers": 1, "window_slice_visits": window, "rows": rows}


def soc_leg(args):
    """SOC-Hubbard (Rashba lambda = 0.5, U/t = -4, n = 1): local, delayed and
    block force-bias updates on forward windows of one walker, per lattice size."""
    import torch
    import synth
    from paper_2506_09611_amd import SocChain, Scheme, soc_batch_forward_window
    rows = []
    for L in [int(x) for x in args.soc_sizes.split(",") if x]:
        N = L * L
        p = synth.make_soc_problem(L, N, -4.0, lam=0.5, dtau=0.05, n_slices=2 * args.soc_window,
                                   stab_every=args.soc_window, perturb=1e-3,
                                   seed=synth.SEED_BASE + 600 + L)
        base = None
        ks = [int(x) for x in args.soc_k.split(",") if x]
        bs = [int(x) for x in args.soc_b.split(",") if x]
        runs = ([] if args.soc_skip_local else [("local", 1)]) + [("delayed", k) for k in ks] \
            + [("block", b) for b in bs]
        for name, k in runs:
            sc = {"local": Scheme.LOCAL, "delayed": Scheme.DELAYED,
                  "block": Scheme.BLOCK_FB}[name]
            c = SocChain(p.hopping, p.trial, p.U, p.dtau, p.n_slices, p.stab_every, p.seed,
                         scheme=sc, k=k, timing=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = c.forward_window(args.soc_window)
            torch.cuda.synchronize()
            w = time.perf_counter() - t0
            fu = args.soc_window * N
            row = {"L": L, "n_e": N, "scheme": name, "k": k,
                   "s_window": w, "field_updates_per_s": fu / w,
                   "update_only": fu / st["t_update_s"] if st["t_update_s"] > 0 else None,
                   "acceptance": st["accepted"] / max(1, st["proposed"])}
            if name == "local":
                base = row
            if base is not None:
                row["speedup_vs_local"] = (row["field_updates_per_s"]
                                           / base["field_updates_per_s"])
                row["update_speedup_vs_local"] = (row["update_only"] / base["update_only"]
                                                  if row["update_only"] and base["update_only"]
                                                  else None)
            log("soc", row)
            rows.append(row)
            c.close()
            del c
            torch.cuda.empty_cache()
        if args.soc_batch > 1 and ks:
            # the same window for a batch of walkers (pqmc_soc_batch_forward_window)
            k = ks[-1]
            cs = [SocChain(p.hopping, p.trial, p.U, p.dtau, p.n_slices, p.stab_every, p.seed,
                           walker_id=w, scheme=Scheme.DELAYED, k=k)
                  for w in range(args.soc_batch)]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            soc_batch_forward_window(cs, args.soc_window)
            torch.cuda.synchronize()
            w = time.perf_counter() - t0
            one = next((r for r in rows if r["L"] == L and r["scheme"] == "delayed"
                        and r["k"] == k), None)
            row = {"L": L, "n_e": N, "scheme": "delayed", "k": k, "walkers": args.soc_batch,
                   "s_window": w,
                   "field_updates_per_s": args.soc_batch * args.soc_window * N / w}
            if one is not None:
                row["speedup_vs_one_walker"] = row["field_updates_per_s"] / one["field_updates_per_s"]
            log("soc batch", row)
            rows.append(row)
            for c in cs:
                c.close()
            del cs
            torch.cuda.empty_cache()
    return {"model": "Rashba SOC-Hubbard, lambda/t = 0.5, U/t = -4, n = 1, dtau = 0.05, "
                     "one walker (batched rows: pqmc_soc_batch_forward_window), complex128",
            "window_slice_visits": args.soc_window, "rows": rows}


def mixed_energy(H0, Gu, Gd, U):
    """Mixed-estimate energy of the Hubbard Hamiltonian from the two spin
    sectors' G (G_ij = <c_i c+_j>, so <c+_i c_j> = delta_ij - G_ji)."""
    import numpy as np
    nu, nd = 1.0 - np.diag(Gu), 1.0 - np.diag(Gd)
    kin = sum(np.trace(H0) - np.sum(H0 * G.T) for G in (Gu, Gd))
    return float(kin + U * np.sum(nu * nd - 0.5 * (nu + nd))), float(np.mean(nu * nd))


def c4_leg(args):
    """Batched walkers with the precision form: 64 walkers of 24x24 (N=576,
    N_sigma=288, U/t=6) and 64 of 12x12 (N=144, N_sigma=72, U/t=6), four of
    each in every batch of 8 (lattices of two sizes in one launch), 16 batches
    on 16 HIP streams, delayed k=32 with the float32 flush (float64 ratios,
    QR and G every 10 slices), two whole sweeps (M=400), the second timed;
    then the same with every sweep one captured HIP graph per batch, and the
    same walkers in float64.  Reports jobs/s (a job = 64 walkers x 1 sweep of
    one lattice) and the mean energy and double occupancy of each job's
    walkers after the second sweep with their standard errors (independent
    chains)."""
    import dataclasses
    import numpy as np
    import torch
    import synth
    from paper_2506_09611_amd import Chain, Scheme, multi_sweep
    p24 = synth.make_problem(24, 288, 288, 6.0, perturb=1e-3, seed=synth.SEED_BASE + 4)
    p12 = synth.make_problem(12, 72, 72, 6.0, perturb=1e-3, seed=synth.SEED_BASE + 5)
    out = {"workload": "64 walkers of 24x24 (N=576, N_sigma=288) + 64 of 12x12 (N=144, "
                       "N_sigma=72), U/t=6, dtau=0.05, M=400, k_tau=10, seeded 1e-3 bond "
                       "perturbation; 16 batches of 4+4 mixed walkers on 16 streams; delayed k=32"}
    for form, fp32, graph in (("fp32", True, False), ("fp32_graph", True, True),
                              ("fp64", False, False)):
        streams = [torch.cuda.Stream() for _ in range(16)]
        chains, jobs = [], []
        for si, st in enumerate(streams):
            for j, q in enumerate((p24, p12)):
                for w in range(4):
                    qq = dataclasses.replace(q, walker_id=si * 4 + w)
                    chains.append(Chain(qq.hopping, qq.trial_up, qq.trial_dn, qq.U, qq.dtau,
                                        qq.n_slices, qq.stab_every, qq.seed, qq.walker_id,
                                        scheme=Scheme.DELAYED, k=32, fp32=fp32, stream=st))
                    if graph:
                        chains[-1].set_opts(Scheme.DELAYED, k=32, graph=True)
                    jobs.append(j)
        torch.cuda.synchronize()
        # sweep 1 (with the graph form, its capture), then the timed sweep 2
        t0 = time.perf_counter()
        multi_sweep(chains, 1)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        stats = multi_sweep(chains, 1)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        fu = 64 * 2 * 400 * (576 + 144)
        rec = {"s_per_sweep": dt, "first_sweep_s": t1 - t0, "jobs_per_s": 2.0 / dt,
               "field_updates_per_s": fu / dt,
               "acceptance": sum(x["accepted"] for x in stats) / sum(x["proposed"] for x in stats),
               "max_stab_drift": max(x["max_stab_drift"] for x in stats)}
        for j, (q, name) in enumerate(((p24, "24x24"), (p12, "12x12"))):
            ed = [mixed_energy(q.hopping, c.green(0), c.green(1), q.U)
                  for c, jj in zip(chains, jobs) if jj == j]
            e = np.array([x[0] for x in ed]) / q.n_sites
            d = np.array([x[1] for x in ed])
            rec[name] = {"energy_per_site": float(e.mean()),
                         "energy_per_site_stderr": float(e.std(ddof=1) / np.sqrt(len(e))),
                         "double_occupancy": float(d.mean()),
                         "double_occupancy_stderr": float(d.std(ddof=1) / np.sqrt(len(d)))}
        if graph:   # captured sweeps are bit for bit the launched ones
            rec["bitwise_equal_to_launched"] = all(
                rec[n] == out["fp32"][n] for n in ("24x24", "12x12"))
        out[form] = rec
        log("c4", form, rec)
        for c in chains:
            c.close()
        del chains
        torch.cuda.empty_cache()
    out["fp32_speedup"] = out["fp64"]["s_per_sweep"] / out["fp32"]["s_per_sweep"]
    out["graph_speedup"] = out["fp32"]["s_per_sweep"] / out["fp32_graph"]["s_per_sweep"]
    for name in ("24x24", "12x12"):
        a, b = out["fp32"][name], out["fp64"][name]
        out[f"{name}_energy_difference_in_stderr"] = abs(
            a["energy_per_site"] - b["energy_per_site"]) / np.hypot(
            a["energy_per_site_stderr"], b["energy_per_site_stderr"])
    out["note"] = ("the float32 and float64 chains are independent (their decisions part "
                   "where a ratio lies within the float32 error of u); the per-proposal "
                   "error statement on identical decisions is tests/test_gpu_precision.py")
    return out


def serve_leg(args, rate):
    """Jobs of mixed lattice sizes and couplings arriving as a Poisson stream
    of `rate` jobs/s, served by the continuous-batching server under an HBM
    budget."""
    import numpy as np
    import synth
    from paper_2506_09611_amd import Scheme
    from paper_2506_09611_amd.serving import GpuBackend, Job, Server, poisson_arrivals
    Ls = [int(x) for x in args.serve_sizes.split(",")]
    Us = [2.0, 4.0, 8.0]
    seed = synth.SEED_BASE + 500
    gen = np.random.Generator(np.random.Philox(key=[seed, 0x4D4958]))
    arrivals = poisson_arrivals(args.serve_jobs, rate, seed)
    probs, jobs = {}, []
    for i in range(args.serve_jobs):
        L, U = Ls[gen.integers(len(Ls))], Us[gen.integers(len(Us))]
        soc = args.serve_soc > 0 and gen.random() < args.serve_soc
        if (L, U, soc) not in probs:
            if soc:   # Rashba lambda = 0.5 at n = 1; the spin-s^y decoupling needs U < 0
                probs[(L, U, soc)] = synth.make_soc_problem(
                    L, L * L, -U, lam=0.5, n_slices=args.serve_slices, stab_every=10,
                    perturb=1e-3, seed=seed + 100 + L)
            else:
                probs[(L, U, soc)] = synth.make_problem(L, L * L // 2, L * L // 2, U,
                                                        n_slices=args.serve_slices,
                                                        stab_every=10, perturb=1e-3,
                                                        seed=seed + L)
        p = probs[(L, U, soc)]
        jobs.append(Job(job_id=i, arrival=float(arrivals[i]), hopping=p.hopping,
                        trial_up=p.trial if soc else p.trial_up,
                        trial_dn=None if soc else p.trial_dn, U=p.U, dtau=p.dtau,
                        n_slices=p.n_slices, stab_every=p.stab_every, seed=seed + 1 + i,
                        n_walkers=args.serve_walkers, n_sweeps=args.serve_sweeps,
                        scheme=Scheme.DELAYED, k=16 if soc else args.k, keep_green=False,
                        soc=soc))
    budget = int(args.serve_budget_gb * 1e9) if args.serve_budget_gb > 0 \
        else GpuBackend.default_budget()
    log(f"serving {len(jobs)} jobs at {rate}/s, budget {budget / 1e9:.2f} GB")
    rep = Server(GpuBackend(lanes=args.serve_lanes), budget).run(jobs)
    out = rep.summary()
    fu = sum(j.n_walkers * j.n_sweeps * 2 * j.n_slices * j.n_sites for j in jobs)
    out.update({
        "arrival_rate_jobs_per_s": rate,
        "field_updates_per_s": fu / rep.makespan_s if rep.makespan_s > 0 else None,
        "soc_jobs": sum(j.soc for j in jobs),
        "scale": f"{args.serve_jobs} of the 512 jobs of the full mix, M={args.serve_slices} "
                 f"of 400 (2 Theta = {args.serve_slices * 0.05:g} of 20), "
                 f"{args.serve_walkers} of 16 walkers per job",
        "mix": f"L in {{{args.serve_sizes}}} uniform, U/t in {{2,4,8}}, half filling; a "
               f"fraction {args.serve_soc} of the jobs Rashba (lambda/t = 0.5, U/t in "
               f"{{-2,-4,-8}}, n = 1, delayed k = 16), "
               f"{args.serve_walkers} walkers x {args.serve_sweeps} sweeps per job, "
               f"M={args.serve_slices}, k_tau=10, delayed k={args.k}, FCFS admission by "
               f"workspace bytes, batches of up to 8 walkers re-formed every sweep, "
               f"{args.serve_lanes} concurrent lanes"})
    log("serving", out)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scheme", default="delayed", choices=["local", "local_g", "delayed", "block"])
    ap.add_argument("--k", type=int, default=32, help="delay rank (0: the autotuner's choice)")
    ap.add_argument("--b", type=int, default=16)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--walkers", type=int, default=8,
                    help="independent walkers swept together in one batch (1..8)")
    ap.add_argument("--streams", type=int, default=2,
                    help="batches of --walkers walkers, one per HIP stream, run concurrently")
    ap.add_argument("--table", default="delayed:8,16,32,64,128;block:1,4,16,64",
                    help="single-walker scheme table timed on forward windows ('' for none)")
    ap.add_argument("--table-window", type=int, default=20,
                    help="slice visits per table entry")
    ap.add_argument("--no-fp32", action="store_true",
                    help="skip the precision-form (float32 T and flush) run of the batch")
    ap.add_argument("--no-single", action="store_true",
                    help="skip the one-walker run of the headline scheme")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized device buffer three times (the reference "
                         "kernel for scaling traffic counters) and exit")
    ap.add_argument("--compare", default="local,local_g,block",
                    help="other schemes timed beside the headline one ('' for none)")
    ap.add_argument("--local-window", type=int, default=10,
                    help="slice visits of the per-site-launch local form timed beside the "
                         "persistent one (0: skip it)")
    ap.add_argument("--u8", action="store_true", default=True,
                    help="also sweep the headline batch at U/t = 8 (the second coupling of "
                         "the 40x40 workload)")
    ap.add_argument("--no-u8", dest="u8", action="store_false")
    ap.add_argument("--no-c4", action="store_true",
                    help="skip the batched precision-form leg (24x24 + 12x12 walkers)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--autotune", default="8,16,32,64,128",
                    help="delay ranks the autotuner times on the headline batch, then the flush "
                         "kernel's tile chunks at the chosen rank ('' to skip)")
    ap.add_argument("--soc-sizes", default="8,16,24",
                    help="lattice sides of the SOC-Hubbard table ('' for none)")
    ap.add_argument("--soc-k", default="8,16,32", help="delay ranks of the SOC table")
    ap.add_argument("--soc-b", default="4,16",
                    help="block sizes of the SOC block force-bias rows (empty: none)")
    ap.add_argument("--soc-skip-local", action="store_true",
                    help="leave the local update out of the SOC table (profiling runs)")
    ap.add_argument("--soc-batch", type=int, default=8,
                    help="walkers of the batched SOC row per lattice size (1: none)")
    ap.add_argument("--soc-window", type=int, default=10,
                    help="forward slice visits per SOC table entry (also k_tau)")
    ap.add_argument("--serve-jobs", type=int, default=32,
                    help="jobs of the serving leg (0 = skip it)")
    ap.add_argument("--serve-rate", default="1,16",
                    help="Poisson arrival rates, jobs/s, one serving run each (comma list)")
    ap.add_argument("--serve-sizes", default="8,12,16,24,32", help="lattice sides L of the mix")
    ap.add_argument("--serve-walkers", type=int, default=16)
    ap.add_argument("--serve-soc", type=float, default=0.5,
                    help="fraction of serving jobs on the Rashba SOC model")
    ap.add_argument("--serve-lanes", type=int, default=4,
                    help="concurrent batches per serving step, one HIP stream each")
    ap.add_argument("--serve-sweeps", type=int, default=1)
    ap.add_argument("--serve-slices", type=int, default=20, help="M of the serving jobs")
    ap.add_argument("--serve-budget-gb", type=float, default=64.0,
                    help="HBM budget of the admitted walkers (0 = 90%% of free memory)")
    ap.add_argument("--tile-chunks", type=int, default=1,
                    help="column chunks per row strip of the flush kernel for the batched "
                         "walkers (1: one per strip, the pipelined strip kernel for groups of "
                         "17-32 sites; 0: the library default of two)")
    ap.add_argument("--ktime-window", type=int, default=10,
                    help="forward slice visits instrumented per kernel after the timed sweeps")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU (walkers are batched on it); --gpus must be 1"}))
        sys.exit(2)

    import torch
    import synth
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration > 0:
        n = args.copy_calibration << 20
        x = torch.zeros(n, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        log(f"copied {args.copy_calibration} MiB x 3")
        return
    p = synth.workload(args.workload)
    N, M = p.n_sites, p.n_slices
    per_sweep = 2 * M * N
    log(f"workload {args.workload}: N={N} N_sigma={p.n_up} M={M}; creating {args.scheme}")

    import dataclasses
    from paper_2506_09611_amd import batch_forward_window
    W, S = args.walkers, args.streams
    if not (1 <= W <= 8 and 1 <= S <= 8):
        ap.error("--walkers and --streams must be 1..8")
    streams = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(S - 1)]
    tuned = None
    if args.autotune and args.scheme == "delayed":
        from paper_2506_09611_amd.autotune import tune_delay
        r = tune_delay(p.hopping, p.trial_up, p.trial_dn, p.U, p.dtau, p.stab_every,
                       candidates=[int(x) for x in args.autotune.split(",")], walkers=W)
        tuned = {"k": r.k, "update_ms_per_slice_visit":
                 {str(k): 1e3 * v for k, v in sorted(r.update_s_per_slice.items())},
                 "tile_chunks": r.tile_chunks, "chunks_update_ms_per_slice_visit":
                 {str(c): 1e3 * v for c, v in sorted(r.chunk_s_per_slice.items())},
                 "walkers": W, "window_slice_visits": p.stab_every}
        log("autotune", tuned)
        torch.cuda.empty_cache()
    if args.k == 0:
        if tuned is None:
            ap.error("--k 0 needs the delayed scheme and --autotune candidates")
        args.k = tuned["k"]
        if args.tile_chunks == 0:
            args.tile_chunks = tuned["tile_chunks"]
    chains = make_walkers(p, args.scheme, args.k, args.b, W, streams,
                          tile_chunks=args.tile_chunks)
    ch = chains[0]
    if args.steps > 0:
        dt, agg = time_sweeps(chains, args.steps, args.warmup)
        value = S * W * args.steps * per_sweep / dt
        # update phase of the first batch (its own events; the batches overlap)
        upd = W * args.steps * per_sweep / agg["t_update_s"] if agg["t_update_s"] > 0 else None
        acc = agg["accepted"] / max(1, agg["proposed"])
    else:   # profiling runs: no timed sweeps, only the instrumented window below
        dt, agg, value, upd, acc = 0.0, {"low_margin": 0, "t_update_s": 0.0, "t_prop_s": 0.0,
                                         "t_stab_s": 0.0}, 0.0, None, 0.74
    # per-kernel device time, live on the library's stream: an instrumented
    # forward window after the timed sweeps
    ch.set_opts(ch.scheme, ch.k, ch.b, ktime=True)
    if args.ktime_window > 0:   # the first batch alone, as in the profiled runs
        kst = batch_forward_window(chains[:W], args.ktime_window)
        if args.steps == 0:     # profiling runs: the window's own acceptance
            acc = sum(x["accepted"] for x in kst) / max(1, sum(x["proposed"] for x in kst))
    ktimes = ch.kernel_times()
    roof = roofline(p, args.scheme, args.k, args.b, acc, ktimes, walkers=W)
    # the rank-n_A flush with the next group's panels, on MFMA (delayed / block)
    roof_flush = roofline(p, args.scheme, args.k, args.b, acc, ktimes, "tile", walkers=W)
    for r in (roof, roof_flush):
        if r is not None:
            r["traffic"] = measured_traffic(r["kernel"], args.scheme, args.k, W, args.workload,
                                            args.tile_chunks)
    if args.steps > 0:
        log(f"{args.scheme}: {dt / args.steps:.3f} s/sweep, {value:.4g} fu/s, "
            f"update-only {upd:.4g}")
    log("kernel times", {c: (round(v[0] * 1e3, 3), v[1]) for c, v in ktimes.items()})
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "field-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps if args.steps else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "40x40 periodic Hubbard, N=1600, N_sigma=800 per spin, U/t=4, dtau=0.05, "
                        "M=400, k_tau=10, seeded 1e-3 bond perturbation"
                        if args.workload == "c3" else args.workload,
            "scheme": args.scheme, "delay_k": args.k, "block_b": args.b, "walkers": S * W,
            "batches": f"{S} x {W} walkers, one HIP stream each, run concurrently",
            "tile_chunks": args.tile_chunks,
        },
        "update_only_field_updates_per_s": upd,
        "acceptance": acc,
        "low_margin": agg["low_margin"],
        "max_stab_drift": agg.get("max_stab_drift"),
        "phase_s_per_sweep": {"update": agg["t_update_s"] / max(1, args.steps),
                              "propagation": agg["t_prop_s"] / max(1, args.steps),
                              "stabilization": agg["t_stab_s"] / max(1, args.steps)},
        "roofline": roof,
        "roofline_flush": roof_flush,
        "kernel_avg_us": {c: 1e6 * v[0] / v[1] for c, v in ktimes.items() if v[1] > 0},
    }
    for c in chains:
        c.close()
    del ch, chains
    torch.cuda.empty_cache()

    # the same scheme on one walker (whole sweeps): the paper's per-chain setting
    if W > 1 and args.steps > 0 and not args.no_single:
        c1 = make_chain(p, args.scheme, args.k, args.b)
        d1, a1 = time_sweeps([c1], 1, 0)
        result["single_chain"] = {
            "walkers": 1, "s_per_sweep": d1, "field_updates_per_s": per_sweep / d1,
            "update_only": per_sweep / a1["t_update_s"] if a1["t_update_s"] > 0 else None,
            "phase_s_per_sweep": {"update": a1["t_update_s"], "propagation": a1["t_prop_s"],
                                  "stabilization": a1["t_stab_s"]}}
        log("single chain", result["single_chain"])
        c1.close()
        del c1
        torch.cuda.empty_cache()

    # the precision form on the same batch (float32 T, flush and panels)
    if args.steps > 0 and not args.no_fp32 and args.scheme != "local":
        cs = make_walkers(p, args.scheme, args.k, args.b, W, streams, fp32=True)
        d32, a32 = time_sweeps(cs, 1, 0)
        result["precision_form"] = {
            "walkers": S * W, "dtype": "f32 T/flush/panels, f64 ratios/QR/inverse",
            "s_per_sweep": d32, "field_updates_per_s": S * W * per_sweep / d32,
            "update_only": W * per_sweep / a32["t_update_s"] if a32["t_update_s"] > 0 else None,
            "speedup_vs_f64": dt / max(1, args.steps) / d32,
            "note": "errors against the float64 oracle: tests/test_gpu_precision.py"}
        log("fp32 form", result["precision_form"])
        for x in cs:
            x.close()
        del cs
        torch.cuda.empty_cache()

    # the same batch at U/t = 8 (c3u8): one whole sweep
    if args.steps > 0 and args.u8 and args.workload == "c3":
        p8 = synth.workload("c3u8")
        cs = make_walkers(p8, args.scheme, args.k, args.b, W, streams)
        d8, a8 = time_sweeps(cs, 1, 0)
        result["u8"] = {"workload": "40x40, U/t=8 (otherwise as the headline)",
                        "walkers": S * W, "s_per_sweep": d8,
                        "field_updates_per_s": S * W * per_sweep / d8,
                        "update_only": W * per_sweep / a8["t_update_s"]
                        if a8["t_update_s"] > 0 else None,
                        "acceptance": a8["accepted"] / max(1, a8["proposed"]),
                        "negative": a8["negative"], "max_stab_drift": a8["max_stab_drift"]}
        log("U/t=8", result["u8"])
        for x in cs:
            x.close()
        del cs
        torch.cuda.empty_cache()

    schemes = {args.scheme: {"s_per_sweep": dt / max(1, args.steps), "field_updates_per_s": value,
                             "update_only": upd, "walkers": S * W}}
    for name in [s for s in args.compare.split(",") if s and s != args.scheme]:
        if name in ("local", "local_g"):
            # the local baselines: one walker, whole sweeps, the persistent
            # kernel (T-form, or the G-form on G itself) over the whole GPU
            c1 = make_chain(p, name)
            d2, a2 = time_sweeps([c1], 1, 0)
            schemes[name] = {"s_per_sweep": d2, "field_updates_per_s": per_sweep / d2,
                             "update_only": per_sweep / a2["t_update_s"]
                             if a2["t_update_s"] > 0 else None,
                             "acceptance": a2["accepted"] / max(1, a2["proposed"]),
                             "max_stab_drift": a2["max_stab_drift"], "walkers": 1,
                             "form": "persistent cooperative kernel, one grid barrier per site"}
            cs = [c1]
            if name == "local" and args.local_window > 0:
                # the per-site-launch form (the one batches of walkers use)
                # (per-launch HIP events on: the per-site kernel against the
                # HBM roofline at the window's own acceptance)
                sl = make_walkers(p, name, args.k, args.b, W, streams[:1])
                for x in sl:
                    x.set_opts(x.scheme, x.k, x.b, site_launches=True, ktime=True)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                kst = batch_forward_window(sl, args.local_window)
                torch.cuda.synchronize()
                w = time.perf_counter() - t0
                acc_l = sum(x["accepted"] for x in kst) / max(1, sum(x["proposed"] for x in kst))
                roof_l = roofline(p, "local", args.k, args.b, acc_l, sl[0].kernel_times(),
                                  "local", walkers=W)
                if roof_l is not None:
                    roof_l["traffic"] = measured_traffic("local", "local", args.k, W,
                                                         args.workload)
                    roof_l["acceptance"] = acc_l
                schemes["local_site_launches"] = {
                    "window_slice_visits": args.local_window, "s_window": w,
                    "field_updates_per_s": W * args.local_window * N / w, "walkers": W,
                    "note": "one launch per site, one batch, forward window, per-launch events",
                    "roofline": roof_l}
                cs += sl
        else:
            cs = make_walkers(p, name, args.k, args.b, W, streams)
            d2, a2 = time_sweeps(cs, 1, 0)
            schemes[name] = {"s_per_sweep": d2, "field_updates_per_s": S * W * per_sweep / d2,
                             "update_only": W * per_sweep / a2["t_update_s"]
                             if a2["t_update_s"] > 0 else None,
                             "acceptance": a2["accepted"] / max(1, a2["proposed"]),
                             "max_stab_drift": a2["max_stab_drift"], "walkers": S * W}
        log(name, schemes[name])
        for x in cs:
            x.close()
        del cs
        torch.cuda.empty_cache()
    for base_name in ("local", "local_g"):
        if base_name in schemes and schemes[base_name]["field_updates_per_s"] > 0:
            base = schemes[base_name]["field_updates_per_s"]
            for v in schemes.values():
                v[f"speedup_vs_{base_name}"] = v["field_updates_per_s"] / base
            if "single_chain" in result:
                result["single_chain"][f"speedup_vs_{base_name}"] = (
                    result["single_chain"]["field_updates_per_s"] / base)
    result["schemes"] = schemes
    if tuned is not None:
        result["autotune"] = tuned
    if args.steps > 0 and not args.no_c4:
        result["batched_precision"] = c4_leg(args)
    if args.table:
        result["table"] = scheme_table(p, args.table, args.table_window)
    if args.soc_sizes:
        result["soc"] = soc_leg(args)
    if args.serve_jobs > 0:
        result["serving"] = [serve_leg(args, float(r)) for r in args.serve_rate.split(",") if r]
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(p, args.scheme, args.k, args.b)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
