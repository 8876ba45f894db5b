#!/usr/bin/env python3
"""Benchmark of the block tensordot hot path on one MI355X.

Workload (timed): the large pairwise contraction -- A and B rank-28 complex
tensors, every dim 2 (2 GiB each in complex64), 14 contracted indices chosen
as a seeded random subset of each operand's axes paired in random order,
unblocked.  One step = plan + permute A + permute B + complex GEMM whose K
loop walks the coupled pairs (fused reduction) + FP64 norm of C, in FP32-4M
(complex64 operands, FP32 MFMA, FP32 accumulation).  The reported value is
useful flops (8*M*N*K) per second of the whole step, inputs already in HBM.

Beside it the same workload runs in FP64 and in split-BF16x3, each with its
error against the oracle on sampled outputs; the sliced 20-qubit amplitude
(4x5 grid, 12 cycles, 4 sliced bonds = 16 slices) gives amplitude latency
percentiles; the oracle is timed on the host on the sampled outputs.

Prints one JSON line on stdout.  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_PEAK = 157.3   # TFLOP/s, dense FP32 MFMA, MI355X
FP64_PEAK = 78.6
BF16_PEAK = 2500.0
# Index of the FP64 Gauss tile (cgemm_f64_3mdl, 64 x 64) in the FP64 tile table.
FP64_GAUSS_TILE = 10
BF16_GAUSS_TILE = 12  # split-BF16 Gauss form, planar operands, eight waves
HBM_PEAK = 8000.0   # GB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if xs else None


def kernel_sha():
    """Hash of the source the profiled GEMM is built from: the shared device
    header (GEMM parameters, output maps, tile order, entry-point macros) and
    the direct-to-LDS FP32 tile with its entry points.  A change there
    invalidates the stored counters."""
    csrc = os.path.join(ROOT, "paper_2201_06620_amd", "csrc")
    with open(os.path.join(csrc, "kcommon.hpp")) as f:
        parts = [f.read()]
    with open(os.path.join(csrc, "gemm_f32_4m.hip")) as f:
        src = f.read()
    i = src.find("// Large-tile FP32-4M with direct-to-LDS staging")
    j = src.find("void launch_tiles_f32_4m(", i) if i >= 0 else -1
    if i < 0 or j < 0:
        return "missing"
    parts.append(src[i:j])
    return hashlib.sha256("".join(parts).encode()).hexdigest()[:16]


def traffic_from_profiles(kernel, per_launch_units):
    """HBM bytes per launch from the committed PMC summary, if still current."""
    path = os.path.join(ROOT, "profiles", "cgemm_f32_rank28_pmc.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_sha():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _make_request(i):
    from workloads import configs
    return configs.config5_request(0, i)


def _size_classes(values):
    """Index lists of the lower, middle and upper third of `values`."""
    order = np.argsort(values, kind="stable")
    n = len(order)
    return {"small": order[: n // 3].tolist(), "medium": order[n // 3: 2 * n // 3].tolist(),
            "large": order[2 * n // 3:].tolist()}


def _latency_summary(res, idx):
    if not idx:
        return None
    lat = [1e3 * res[i]["latency_s"] for i in idx]
    return {"n": len(idx), "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99),
            "mean_queue_ms": 1e3 * float(np.mean([res[i]["queue_s"] for i in idx])),
            "mean_run_ms": 1e3 * float(np.mean([res[i]["run_s"] for i in idx])),
            "p99_queue_ms": percentile([1e3 * res[i]["queue_s"] for i in idx], 99),
            "p99_run_ms": percentile([1e3 * res[i]["run_s"] for i in idx], 99)}


def run_serving(args, torch, rn, log):
    """Requests of the serving workload: seeded random circuits on 30-53-site
    grids, 8-14 cycles, each with 1-64 slices and sliced further until its
    largest intermediate has rank <= 30, complex64 with FP64 slice sums.
    First all requests are queued at once (saturated throughput); then, for
    each load in --serve-loads, the same requests arrive as a Poisson stream
    at that fraction of the saturated rate.  Latency = completion - arrival,
    split into queueing (arrival to admission) and running time, overall and
    per size third (total flops).  A seeded tenth of the requests is checked
    against the oracle, one slice each (see serving_oracle_sample)."""
    import threading
    from concurrent.futures import ProcessPoolExecutor

    t0 = time.time()
    with ProcessPoolExecutor(max_workers=max(1, min(16, os.cpu_count() or 1))) as ex:
        reqs = list(ex.map(_make_request, range(args.serve_requests)))
    log(f"serving: {len(reqs)} requests planned in {time.time() - t0:.1f}s")
    free, total = torch.cuda.mem_get_info()
    budget = int(0.9 * free)
    srv = rn.Server(0, hbm_budget=budget, max_active=args.serve_slots)
    tensors = [[t.astype(np.complex64) for t in w.network.tensors] for w in reqs]
    flops = [w.meta["total_flops"] for w in reqs]

    def submit(i):
        w = reqs[i]
        return srv.submit(tensors[i], w.network.labels, w.path, w.sliced, "fp32_4m")

    # Warm-up (kernel first use), not counted.
    srv.wait(submit(0))
    t = time.perf_counter()
    tickets = [submit(i) for i in range(len(reqs))]
    sat = [srv.wait(tk) for tk in tickets]
    sat_s = time.perf_counter() - t
    thr = len(reqs) / sat_s
    log(f"serving: saturated {thr:.1f} amplitudes/s ({sat_s:.2f} s for {len(reqs)})")
    classes = _size_classes(flops)

    def sweep_loads(loads, tag):
        out = []
        for load in loads:
            lam = load * thr
            # Arrival gaps seeded by the load alone: both admission policies see
            # the same arrival sequence at a given load.
            gaps = np.random.default_rng(2201 + int(round(100 * load))).exponential(
                1.0 / lam, size=len(reqs))
            tk2 = [None] * len(reqs)

            def client():
                for i, g in enumerate(gaps):
                    time.sleep(float(g))
                    tk2[i] = submit(i)

            t = time.perf_counter()
            th = threading.Thread(target=client)
            th.start()
            th.join()
            res = [srv.wait(tk) for tk in tk2]
            el = time.perf_counter() - t
            lat = [1e3 * r["latency_s"] for r in res]
            same = sum(1 for a, b in zip(sat, res) if a["amp"] == b["amp"] and a["status"] == 0)
            entry = {"load": load, "arrival_rate_per_s": lam, "p50_ms": percentile(lat, 50),
                     "p99_ms": percentile(lat, 99), "amplitudes_per_s": len(reqs) / el,
                     "mean_queue_ms": 1e3 * float(np.mean([r["queue_s"] for r in res])),
                     "mean_run_ms": 1e3 * float(np.mean([r["run_s"] for r in res])),
                     "by_size_third": {k: _latency_summary(res, v) for k, v in classes.items()},
                     "identical_to_saturated_run": same,
                     "statuses": sorted(set(r["status"] for r in res))}
            # Achieved rate of the largest tenth of the requests while they ran
            # (each request's flops over its own running time; other requests
            # may have shared the GPU meanwhile).
            top = np.argsort(flops)[-max(1, len(reqs) // 10):]
            entry["largest_tenth_tflops_while_running"] = float(
                sum(flops[i] for i in top) / sum(res[i]["run_s"] for i in top) / 1e12)
            log(f"serving {tag} load {load}: p50 {entry['p50_ms']:.1f} ms, "
                f"p99 {entry['p99_ms']:.1f} ms, {entry['amplitudes_per_s']:.1f}/s")
            out.append(entry)
        return out

    sweep = sweep_loads(args.serve_loads, "smallest-first")
    srv.set_admission("fifo")
    sweep_fifo = sweep_loads([x for x in args.serve_loads if x >= 0.75], "arrival-order")
    srv.set_admission("smallest")
    srv.close()
    hist_sites = {}
    hist_slices = {}
    for w in reqs:
        key = f"{w.meta['sites']}x{w.meta['cycles']}"
        hist_sites[key] = hist_sites.get(key, 0) + 1
        hist_slices[str(1 << len(w.sliced))] = hist_slices.get(str(1 << len(w.sliced)), 0) + 1
    out = {"workload": "amplitude requests for seeded random circuits on 30-53-site grids, 8-14 "
                       "cycles, 1-64 slices each (2^0..2^6) and sliced until the largest "
                       "intermediate rank <= 30, complex64 FP32-4M with FP64 slice sums; "
                       f"HBM-footprint admission, {args.serve_slots} concurrent slots",
           "requests": len(reqs), "saturated_amplitudes_per_s": thr,
           "saturated_seconds": sat_s, "admission": "smallest planned flops first, a request "
                                                    "overtaken 8 times goes next",
           "loads": sweep, "loads_arrival_order_admission": sweep_fifo,
           "total_flops": float(sum(flops)),
           "accepted_sites_x_cycles": dict(sorted(hist_sites.items())),
           "slices_per_request": dict(sorted(hist_slices.items(), key=lambda kv: int(kv[0]))),
           "size_thirds_total_flops": {k: float(sum(flops[i] for i in v))
                                       for k, v in classes.items()}}
    return out, reqs


def serving_oracle_sample(args, torch, rn, oracle, reqs, log):
    """e_amp of a seeded tenth of the served requests against the oracle,
    slice-subsampled: each sampled request runs once more through
    rn_contract_network (FP32-4M, the kernels the server runs) with its
    per-slice values returned, and one slice (seeded choice) is compared with
    the oracle's projection of that slice.  A request whose slices cost more
    than --oracle-slice-flops is sliced deeper for the check (more bonds,
    chosen by the same greedy slicer) on both sides, and says so.  Error:
    |a - a_ref| / max(|a_ref|, 2^-(n+S)/2), n sites, S sliced bonds."""
    from workloads import paths
    ctx = rn.Context(0)
    rs = np.random.default_rng(5150)
    pick = sorted(rs.choice(len(reqs), size=max(1, len(reqs) // 10), replace=False).tolist())
    rows = []
    t_or = 0.0
    for i in pick:
        w = reqs[i]
        lab, path = w.network.labels, w.path
        sliced = list(w.sliced)
        mr, fl, _ = paths.path_stats(lab, path, sliced)
        deeper = 0
        while fl > args.oracle_slice_flops and len(sliced) < 14:
            more = paths.greedy_slices(lab, path, 77 + i, n_slices=len(sliced) + 1)
            extra = [x for x in more if x not in sliced]
            if not extra:
                break
            sliced.append(extra[0])
            deeper += 1
            mr, fl, _ = paths.path_stats(lab, path, sliced)
        S = len(sliced)
        ts = [torch.from_numpy(np.ascontiguousarray(t.reshape(-1))).to(torch.complex64).cuda()
              for t in w.network.tensors]
        sl = torch.zeros(2 << S, dtype=torch.float64, device="cuda")
        ctx.contract_network(ts, lab, path, sliced, "fp32_4m", slices=sl)
        torch.cuda.synchronize()
        got = sl.cpu().numpy().view(np.complex128)
        s = int(rs.integers(0, 1 << S))
        t = time.perf_counter()
        ref = oracle.contract_network_slices(w.network.tensors, lab, path, sliced, [s])[0]
        t_or += time.perf_counter() - t
        n = w.meta["sites"]
        err = abs(got[s] - ref) / max(abs(ref), 2.0 ** (-(n + S) / 2))
        rows.append({"request": i, "sites": n, "cycles": w.meta["cycles"],
                     "sliced_served": len(w.sliced), "sliced_for_check": S,
                     "extra_sliced_for_check": deeper, "slice": s,
                     "flops_per_slice_checked": fl, "e_amp": float(err)})
        log(f"serving oracle check: request {i} ({n} sites, {S} sliced, +{deeper} for the "
            f"check) slice {s}: e_amp {err:.2e}")
        del ts, sl
    ctx.close()
    errs = [r["e_amp"] for r in rows]
    return {"sampled": len(rows), "of_requests": len(reqs), "mode": "fp32_4m",
            "tolerance": 1e-5, "max_e_amp": float(max(errs)),
            "median_e_amp": float(np.median(errs)), "oracle_seconds": t_or,
            "how": "one seeded slice per sampled request, GPU per-slice value vs the oracle's "
                   "projection of that slice; requests above the per-slice flop cap sliced "
                   "deeper for the check on both sides",
            "rows": rows}


def run_weak_share(args, torch, rn, log):
    """Weak-scaling workload of the paper's evaluation (Section V.C), one
    device's share at the real block shape: U (m x k) . V (n x k)^T with
    blocks m_b = n_b = 2^14, k_b = 2^13, complex64, B_m x B_n = 8 x 6 output
    blocks (Table I, one node) and B_k coupled pairs.  B_n = 6 is not a power
    of two, so the share runs as two contractions sharing U: 4 and 2 output
    block columns.

    placement "hbm": both operands resident in HBM and the pairs fused into
    one K loop (every pair's blocks in memory at once, the Eq. 1 regime).
    placement "streamed": operands in pinned host memory, pairs copied in as
    needed and added into the HBM output blocks (the commutative reduction,
    Eq. 2 per block in flight).  Prints one JSON line per run.
    """
    ctx = rn.Context(0)
    dev = "cuda:0"
    mb_bits, nb_inner, kb_inner = args.weak_block_bits
    oracle = None
    if not args.no_cpu_baseline:
        import oracle

    def gen_device(n, seed):
        g = torch.Generator(device=dev)
        g.manual_seed(seed)
        return torch.randn(n, dtype=torch.complex64, device=dev, generator=g)

    def gen_pinned(n, seed):
        host = torch.empty(n, dtype=torch.complex64, pin_memory=True)
        g = torch.Generator(device=dev)
        g.manual_seed(seed)
        chunk = 1 << 27
        for o in range(0, n, chunk):
            m = min(chunk, n - o)
            host[o:o + m].copy_(torch.randn(m, dtype=torch.complex64, device=dev, generator=g))
        torch.cuda.synchronize()
        return host

    def shapes(bm_bits, bn_bits, bk_bits, blocked):
        # Axes: U = [m block bits | m inner | k block bits | k inner]; for a
        # blocked (block-major) store the block bits carry grid 2.
        ua = bm_bits + mb_bits + bk_bits + kb_inner
        va = bn_bits + nb_inner + bk_bits + kb_inner
        g = 2 if blocked else 1
        gu = [g] * bm_bits + [1] * mb_bits + [g] * bk_bits + [1] * kb_inner
        gv = [g] * bn_bits + [1] * nb_inner + [g] * bk_bits + [1] * kb_inner
        ax_u = list(range(bm_bits + mb_bits, ua))
        ax_v = list(range(bn_bits + nb_inner, va))
        return [2] * ua, gu, [2] * va, gv, ax_u, ax_v

    def sample_check(c_flat, u_rows, v_rows, m_total, n_total, k_total, blocked, bn_bits):
        # A few outputs recomputed in complex128 from the operand rows: by the
        # oracle (the contraction of the two rows over all their axes) in the
        # CPU-baseline leg, else by numpy's dot product.
        rs = np.random.default_rng(13)
        worst = 0.0
        kb = int(k_total).bit_length() - 1
        for _ in range(4):
            i = int(rs.integers(0, m_total))
            j = int(rs.integers(0, n_total))
            ur = u_rows(i).astype(np.complex128)
            vr = v_rows(j).astype(np.complex128)
            if oracle is not None:
                ref = complex(oracle.tensordot(ur.reshape([2] * kb), vr.reshape([2] * kb),
                                               list(range(kb)), list(range(kb))))
            else:
                ref = np.dot(ur, vr)
            if blocked:
                bi, ii = i >> mb_bits, i & ((1 << mb_bits) - 1)
                bj, jj = j >> nb_inner, j & ((1 << nb_inner) - 1)
                off = ((bi << bn_bits) + bj) * (1 << (mb_bits + nb_inner)) + (ii << nb_inner) + jj
            else:
                off = i * n_total + j
            got = complex(c_flat[off].item())
            worst = max(worst, abs(got - ref) / (np.linalg.norm(ur) * np.linalg.norm(vr)))
        return worst

    bm_bits = 3
    results = []
    for placement, bk_list, sub in (("hbm", args.weak_bk, None),
                                    ("streamed", args.stream_bk, None),
                                    ("streamed", args.stream_sub_bk, (0, 1)),
                                    ("hbm", args.stream_sub_bk, (0, 1))):
        for bk in bk_list:
            bk_bits = int(bk).bit_length() - 1
            rows_bits = bm_bits if sub is None else sub[0]
            col_splits = [2, 1] if sub is None else [sub[1]]  # 4 + 2 columns, or a sub-grid
            blocked = placement == "streamed"
            m_total = 1 << (rows_bits + mb_bits)
            k_total = 1 << (bk_bits + kb_inner)
            log(f"weak share: placement={placement} B_k={bk} rows={1 << rows_bits} "
                f"cols={sum(1 << c for c in col_splits)}")
            u_n = m_total * k_total
            seed = 5000 + bk
            u = gen_pinned(u_n, seed) if blocked else gen_device(u_n, seed)
            total_fl = 0.0
            total_s = 0.0
            dev_bytes = u_n * 8 if not blocked else 0
            h2d = 0.0
            ws_max = 0
            worst = 0.0
            for ci, bn_bits in enumerate(col_splits):
                du, gu, dv, gv, ax_u, ax_v = shapes(rows_bits, bn_bits, bk_bits, blocked)
                n_total = 1 << (bn_bits + nb_inner)
                v_n = n_total * k_total
                v = gen_pinned(v_n, seed * 10 + ci) if blocked else gen_device(v_n, seed * 10 + ci)
                c = torch.empty(m_total * n_total, dtype=torch.complex64, device=dev)
                if blocked:
                    _, _, ws, fl, hb = ctx.plan_streamed(du, gu, dv, gv, ax_u, ax_v, "fp32_4m")
                    h2d += hb
                else:
                    _, _, ws, fl = ctx.plan_block_tensordot(du, gu, dv, gv, ax_u, ax_v, "fp32_4m")
                    dev_bytes += v_n * 8
                wsb = torch.empty(max(ws, 1), dtype=torch.uint8, device=dev)
                ws_max = max(ws_max, ws)
                dev_bytes += m_total * n_total * 8
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                if blocked:
                    ctx.block_tensordot_streamed(u, du, gu, v, dv, gv, ax_u, ax_v, "fp32_4m",
                                                 out=c, workspace=wsb)
                else:
                    ctx.block_tensordot(u, du, gu, v, dv, gv, ax_u, ax_v, "fp32_4m", out=c,
                                        workspace=wsb)
                e1.record()
                torch.cuda.synchronize()
                sec = e0.elapsed_time(e1) / 1e3
                total_s += sec
                total_fl += fl
                log(f"  columns 2^{bn_bits}: {sec:.2f} s, {fl / sec / 1e12:.1f} TFLOP/s")

                def u_row(i, u=u, blocked=blocked, k_total=k_total):
                    if not blocked:
                        return u[i * k_total:(i + 1) * k_total].cpu().numpy()
                    # Block-major: row i of block row bi spans B_k blocks.
                    bi, ii = i >> mb_bits, i & ((1 << mb_bits) - 1)
                    kb = 1 << kb_inner
                    blk = (1 << mb_bits) * kb
                    parts = [u[((bi << bk_bits) + q) * blk + ii * kb:
                               ((bi << bk_bits) + q) * blk + (ii + 1) * kb]
                             for q in range(1 << bk_bits)]
                    return torch.cat(parts).cpu().numpy()

                def v_row(j, v=v, blocked=blocked, k_total=k_total):
                    if not blocked:
                        return v[j * k_total:(j + 1) * k_total].cpu().numpy()
                    bj, jj = j >> nb_inner, j & ((1 << nb_inner) - 1)
                    kb = 1 << kb_inner
                    blk = (1 << nb_inner) * kb
                    parts = [v[((bj << bk_bits) + q) * blk + jj * kb:
                               ((bj << bk_bits) + q) * blk + (jj + 1) * kb]
                             for q in range(1 << bk_bits)]
                    return torch.cat(parts).cpu().numpy()

                worst = max(worst, sample_check(c, u_row, v_row, m_total, n_total, k_total,
                                                blocked, bn_bits))
                del v, c, wsb
                torch.cuda.empty_cache()
            del u
            torch.cuda.empty_cache()
            if blocked and hasattr(torch._C, "_host_emptyCache"):
                torch._C._host_emptyCache()  # return the pinned staging to the system
            kb_ = 1 << kb_inner
            m_b = n_b = 1 << mb_bits
            line = {"mode": "weak_share", "placement": placement, "B_k": bk,
                    "B_m": 1 << rows_bits, "B_n": sum(1 << c for c in col_splits),
                    "block": [m_b, n_b, kb_], "dtype": "c64 (fp32_4m)",
                    "seconds": round(total_s, 3), "tflops": round(total_fl / total_s / 1e12, 2),
                    "useful_flops": total_fl,
                    "device_bytes": dev_bytes + ws_max,
                    "eq1_task_elems": bk * kb_ * (m_b + n_b) + m_b * n_b,
                    "eq2_task_elems": kb_ * (m_b + n_b) + m_b * n_b,
                    "h2d_bytes": h2d, "h2d_GBps": round(h2d / total_s / 1e9, 2) if h2d else None,
                    "max_rel_err_sampled": worst,
                    "reference": "numpy" if oracle is None else "oracle"}
            print(json.dumps(line), flush=True)
            results.append(line)
    ctx.close()
    return results


def host_info():
    """CPU model and core counts of the host (for the CPU-baseline figures)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = None
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity_cores": aff}


def network_roofline(labels, path, sliced, es, peak_tflops):
    """Useful flops, algorithmic bytes and roofline time of a sliced network
    as the library runs it: every step runs once per value combination of the
    sliced bonds its operands depend on (slice-independent parts once), on
    operands with the sliced labels projected out; per step
    F = 8 * 2^|labels(a) | labels(b)| and B = es * (|a| + |b| + |out|), and
    the roofline time is the sum over steps of max(F / peak, B / HBM)."""
    sl = set(sliced)
    live = [frozenset(l) - sl for l in labels]
    deps = [frozenset(l) & sl for l in labels]
    F = B = T = 0.0
    for a, b in path:
        la, lb = live[a], live[b]
        out = la ^ lb
        d = deps[a] | deps[b]
        mult = float(1 << len(d))
        f = 8.0 * (1 << len(la | lb)) * mult
        by = es * float((1 << len(la)) + (1 << len(lb)) + (1 << len(out))) * mult
        F += f
        B += by
        T += max(f / (peak_tflops * 1e12), by / (HBM_PEAK * 1e9))
        live.append(out)
        deps.append(d)
    return F, B, T


def run_config1(ctx, torch, oracle, parity, reps, log):
    """Workload 1 (rank-16 x rank-16 complex, 8 contracted axes, first three
    axes of each operand split in two: 64 coupled block pairs of 32 x 256 x
    32): latency per call (plan + relayouts + GEMM, HIP-event and host-wall
    time over `reps` calls after 3 warm-ups, synchronised each call; and the
    same contraction as a prepared, graph-replayed call) and the error
    against the oracle, in every mode."""
    from workloads import configs
    p = configs.config1()
    t = time.perf_counter()
    ref, _, _ = oracle.block_tensordot(p.a.data, p.a.dims, p.a.grid, p.b.data, p.b.dims,
                                       p.b.grid, p.axes_a, p.axes_b)
    t_single = time.perf_counter() - t
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    t = time.perf_counter()
    ref_omp, _, _ = oracle.block_tensordot(p.a.data, p.a.dims, p.a.grid, p.b.data, p.b.dims,
                                           p.b.grid, p.axes_a, p.axes_b, openmp=True)
    t_omp = time.perf_counter() - t
    absprod = parity.abs_product_blocked(p)
    K = 2 ** p.k
    flops = 8.0 * 2 ** 24
    out = {"workload": "rank-16 x rank-16 complex, A's last 8 axes with B's first 8 in seeded "
                       "order, first three axes of each operand split in two (64 block pairs "
                       "of 32 x 256 x 32); one call = plan + relayouts + fused-pair GEMM",
           "useful_flops": flops, "reps": reps}
    for mode in ("fp64", "fp32_4m", "fp32_3m", "bf16x3"):
        dt = torch.complex128 if mode == "fp64" else torch.complex64
        a = torch.from_numpy(p.a.data).to(dt).cuda()
        b = torch.from_numpy(p.b.data).to(dt).cuda()
        cd, cg, ws, _ = ctx.plan_block_tensordot(p.a.dims, p.a.grid, p.b.dims, p.b.grid,
                                                 p.axes_a, p.axes_b, mode)
        c = torch.empty(2 ** 16, dtype=dt, device="cuda")
        wsb = torch.empty(max(ws, 1), dtype=torch.uint8, device="cuda")
        host, ev = [], []
        for it in range(3 + reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            t = time.perf_counter()
            e0.record()
            ctx.block_tensordot(a, p.a.dims, p.a.grid, b, p.b.dims, p.b.grid, p.axes_a,
                                p.axes_b, mode, out=c, workspace=wsb)
            e1.record()
            torch.cuda.synchronize()
            if it >= 3:
                host.append(1e6 * (time.perf_counter() - t))
                ev.append(1e3 * e0.elapsed_time(e1))
        r = parity.report(c.cpu().numpy().astype(np.complex128), ref, absprod, K, mode)
        # The same contraction as a prepared call (descriptors and plan built
        # once, a one-problem batch replayed as a HIP graph on a side stream):
        # the latency of repeated calls on one shape.
        c2 = torch.empty_like(c)
        pb = ctx.prepare_batch([(a, p.a.dims, p.a.grid, b, p.b.dims, p.b.grid, p.axes_a,
                                 p.axes_b)], mode, outs=[c2])
        side = torch.cuda.Stream()
        prep = []
        for it in range(3 + reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            with torch.cuda.stream(side):
                pb.run()
            side.synchronize()
            if it >= 3:
                prep.append(1e6 * (time.perf_counter() - t))
        r2 = parity.report(c2.cpu().numpy().astype(np.complex128), ref, absprod, K, mode)
        out[mode] = {"p50_us_host": percentile(host, 50), "p10_us_host": percentile(host, 10),
                     "p90_us_host": percentile(host, 90), "p50_us_gpu_events": percentile(ev, 50),
                     "e_F": r["e_F"], "e_max": r["e_max"], "higham_max": r["higham"],
                     "higham_bound": r["higham_bound"], "tolerance": parity.TOL[mode],
                     "prepared_p50_us_host": percentile(prep, 50),
                     "prepared_e_F": r2["e_F"], "prepared_higham_max": r2["higham"]}
        log(f"config1 {mode}: p50 {out[mode]['p50_us_host']:.1f} us host, "
            f"{out[mode]['p50_us_gpu_events']:.1f} us events, prepared "
            f"{out[mode]['prepared_p50_us_host']:.1f} us, e_F {r['e_F']:.2e}")
        del a, b, c, c2, wsb, pb
    out["oracle"] = {"single_thread_s": t_single,
                     "single_thread_gflops": flops / t_single / 1e9,
                     "openmp_s": t_omp, "openmp_threads": min(threads, 8),
                     "openmp_gflops": flops / t_omp / 1e9,
                     "openmp_note": "output blocks on threads; workload 1 has 8 output blocks, "
                                    "so at most 8 threads have work",
                     "openmp_identical_to_single_thread": bool(np.array_equal(ref, ref_omp))}
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--side-steps", type=int, default=3,
                    help="timed steps for the FP64 and BF16x3 side measurements")
    ap.add_argument("--rank", type=int, default=28)
    ap.add_argument("--k", type=int, default=14)
    ap.add_argument("--amp-requests", type=int, default=40)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sample-blocks", type=int, default=40,
                    help="64 x 64 blocks of C the oracle computes for the CPU baseline")
    ap.add_argument("--config1-reps", type=int, default=30)
    ap.add_argument("--no-side", action="store_true")
    ap.add_argument("--no-batch", dest="batch", action="store_false")
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--serve-slots", type=int, default=4,
                    help="requests the server runs concurrently (1-16)")
    ap.add_argument("--serve-loads", type=lambda x: [float(v) for v in x.split(",") if v],
                    default=[0.25, 0.5, 0.75, 1.0],
                    help="Poisson arrival rates as fractions of the saturated throughput")
    ap.add_argument("--oracle-slice-flops", type=float, default=3e9,
                    help="largest per-slice cost the serving oracle check contracts")
    ap.add_argument("--copy-calib", action="store_true",
                    help="run one plain 1 GiB copy kernel first (HBM counter calibration)")
    ap.add_argument("--weak", action="store_true",
                    help="run only the weak-scaling share (one JSON line per run) and exit")
    ap.add_argument("--weak-bk", type=lambda x: [int(v) for v in x.split(",") if v],
                    default=[2, 4, 8], help="B_k values run with both operands in HBM")
    ap.add_argument("--stream-bk", type=lambda x: [int(v) for v in x.split(",") if v],
                    default=[2], help="B_k values streamed from host memory (8 x 6 blocks)")
    ap.add_argument("--stream-sub-bk", type=lambda x: [int(v) for v in x.split(",") if v],
                    default=[16], help="B_k values run on a 1 x 2 block sub-grid, streamed "
                                       "and in HBM")
    ap.add_argument("--weak-block-bits", type=lambda x: [int(v) for v in x.split(",")],
                    default=[14, 14, 13], help="log2 of m_b, n_b, k_b (a smaller block for "
                                               "quick checks)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the library runs on one GPU; the contraction is not "
                                   "sharded across GPUs (run with --gpus 1)"}))
        return 2

    import torch
    import oracle
    import paper_2201_06620_amd as rn
    from workloads import configs
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import parity  # element-wise error bounds (test infrastructure, CPU side)

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        return 1
    if args.weak:
        run_weak_share(args, torch, rn, log)
        return 0
    ctx = rn.Context(0)
    dev = "cuda:0"

    # ------------------------------------------------------------ inputs
    t0 = time.time()
    p = configs.config3(rank=args.rank, k=args.k)
    log(f"inputs generated in {time.time() - t0:.1f}s: rank {args.rank}, k {args.k}, "
        f"axes_a={p.axes_a} axes_b={p.axes_b}")
    dims = [2] * args.rank
    M = N = 2 ** (args.rank - args.k)
    K = 2 ** args.k
    flops = 8.0 * M * N * K

    # Sampled outputs: --sample-blocks 64 x 64 blocks of C viewed as M x N (row-major C).
    rs = np.random.default_rng(2201)
    sample = []
    for _ in range(args.sample_blocks):
        r0 = int(rs.integers(0, M // 64)) * 64
        c0 = int(rs.integers(0, N // 64)) * 64
        rr, cc = np.meshgrid(np.arange(r0, r0 + 64), np.arange(c0, c0 + 64), indexing="ij")
        sample.append((rr * N + cc).reshape(-1))
    sample = np.concatenate(sample).astype(np.int64)

    def run_mode(mode, steps, warmup, profile):
        dt = torch.complex128 if mode == "fp64" else torch.complex64
        a = torch.from_numpy(p.a.data).to(dt).to(dev)
        b = torch.from_numpy(p.b.data).to(dt).to(dev)
        cd, cg, ws, fl = rn.plan_block_tensordot(dims, None, dims, None, p.axes_a, p.axes_b, mode)
        c = torch.empty(M * N, dtype=dt, device=dev)
        wsb = torch.empty(max(ws, 1), dtype=torch.uint8, device=dev)

        def step():
            ctx.block_tensordot(a, dims, None, b, dims, None, p.axes_a, p.axes_b, mode, out=c,
                                workspace=wsb)
            return ctx.norm2(c, [2] * (2 * (args.rank - args.k)))

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        if profile:
            ctx.profile(True)
            ctx.profile_read()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            nrm = step()
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        kern = ctx.profile_read() if profile else None
        ctx.profile(False)
        got = c[torch.from_numpy(sample).to(dev)].cpu().numpy().astype(np.complex128)
        out = {"ms_per_step": 1e3 * el / steps, "tflops": flops * steps / el / 1e12,
               "norm2_c": float(nrm.item()), "kernels": kern}
        del a, b, c, wsb
        torch.cuda.empty_cache()
        return out, got

    if args.copy_calib:
        x = torch.ones(2 ** 28, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written by one elementwise kernel")
        del x, y

    log("FP32-4M timed run")
    main_res, got32 = run_mode("fp32_4m", args.steps, args.warmup, True)
    log(f"  {main_res['ms_per_step']:.2f} ms/step, {main_res['tflops']:.2f} TFLOP/s; "
        f"kernels {main_res['kernels']}")
    side = {}
    gots = {"fp32_4m": got32}
    if not args.no_side:
        for mode in ("fp32_3m", "bf16x3", "fp64"):
            log(f"{mode} side run")
            r, g = run_mode(mode, args.side_steps, 1, True)
            side[mode] = r
            gots[mode] = g
            log(f"  {r['ms_per_step']:.2f} ms/step, {r['tflops']:.2f} TFLOP/s")
        # FP64 mode with the Gauss GEMM tile (three real products per complex
        # product), an alternative FP64 tile selected through a tune file.
        log("fp64 with the Gauss tile (fp64_gauss) side run")
        with tempfile.TemporaryDirectory() as td:
            tf = os.path.join(td, "fp64_gauss_tune.txt")
            with open(tf, "w") as f:
                f.write("rn_tune 1\n%d %d %d %d %d\n" % (0, args.rank - args.k, args.rank - args.k,
                                                         args.k, FP64_GAUSS_TILE))
            ctx.tune_load(tf)
            r, g = run_mode("fp64", args.side_steps, 1, True)
            ctx.tune_clear()
        side["fp64_gauss"] = r
        gots["fp64_gauss"] = g
        log(f"  {r['ms_per_step']:.2f} ms/step, {r['tflops']:.2f} TFLOP/s")
        # Split BF16 in the Gauss form (planar operands, nine bf16 MFMAs per
        # 16 complex k instead of twelve), selected through a tune file.
        log("bf16x3 with the Gauss tile (bf16x3_gauss) side run")
        with tempfile.TemporaryDirectory() as td:
            tf = os.path.join(td, "bf16_gauss_tune.txt")
            with open(tf, "w") as f:
                f.write("rn_tune 1\n%d %d %d %d %d\n" % (3, args.rank - args.k, args.rank - args.k,
                                                         args.k, BF16_GAUSS_TILE))
            ctx.tune_load(tf)
            r, g = run_mode("bf16x3", args.side_steps, 1, True)
            ctx.tune_clear()
        side["bf16x3_gauss"] = r
        gots["bf16x3_gauss"] = g
        log(f"  {r['ms_per_step']:.2f} ms/step, {r['tflops']:.2f} TFLOP/s")

    # ------------------------------------------------ oracle on the sample
    cpu = None
    ref = None
    absprod = None
    if not args.no_cpu_baseline:
        A = p.a.data.reshape(dims)
        B = p.b.data.reshape(dims)
        log(f"oracle on {sample.size} sampled outputs (single thread)")
        t = time.perf_counter()
        ref = oracle.tensordot_entries(A, B, p.axes_a, p.axes_b, sample)
        el = time.perf_counter() - t
        hi = host_info()
        cpu = {"value": 8.0 * K * sample.size / el / 1e12, "unit": "TFLOP/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{sample.size} output entries ({args.sample_blocks} 64x64 blocks of C) "
                         f"of the same rank-{args.rank} contraction, each a {K}-term complex128 "
                         f"sum; {el:.1f} s",
               "cpu_model": hi["cpu_model"], "nproc": hi["nproc"],
               "affinity_cores": hi["affinity_cores"],
               "extrapolated_full_contraction_s": el / sample.size * M * N,
               "extrapolation_note": "seconds per sampled entry times all M*N entries, one "
                                     "thread (an extrapolation, not a run)"}
        log(f"  {el:.1f}s -> {cpu['value'] * 1e3:.4f} GFLOP/s; full contraction extrapolated "
            f"to {cpu['extrapolated_full_contraction_s'] / 3600:.1f} h")
        absprod = parity.abs_product_entries(A, B, p.axes_a, p.axes_b, sample)

    errors = {}
    if ref is not None:
        for mode, g in gots.items():
            pm = "fp64" if mode.startswith("fp64") else "bf16x3" if mode.startswith("bf16") else mode
            r = parity.report(g, ref, absprod, K, pm)
            errors[mode] = {"e_F": r["e_F"], "e_max": r["e_max"], "higham_max": r["higham"],
                            "higham_bound": r["higham_bound"],
                            "entries_over_bound": r["over_bound"]}
        log(f"sampled errors vs oracle: {errors}")
    config1 = None
    if not args.no_cpu_baseline and args.config1_reps > 0:
        config1 = run_config1(ctx, torch, oracle, parity, args.config1_reps, log)

    # ------------------------------------------- amplitude latency (16 slices)
    amp = None
    side_stream = torch.cuda.Stream()
    if args.amp_requests > 0:
        w = configs.config2()
        lat = {}
        for mode, slice_sum in (("fp64", 0), ("fp32_4m", 0), ("fp64", 1), ("fp32_4m", 1)):
            ctx.set_option("slice_sum", slice_sum)
            dt = torch.complex128 if mode == "fp64" else torch.complex64
            ts = [torch.from_numpy(np.ascontiguousarray(t.reshape(-1))).to(dt).to(dev)
                  for t in w.network.tensors]
            # One circuit, its call prepared once (argument arrays, plan); each
            # request runs on a side stream, so repeats replay a captured graph
            # (first call direct, second captured).
            net = ctx.prepare_network(ts, w.network.labels, w.path, w.sliced, mode)
            fl = net.flops
            ampt = torch.zeros(2, dtype=torch.float64, device=dev)
            torch.cuda.synchronize()
            for _ in range(3):
                net.run(amp=ampt, stream=side_stream)
                side_stream.synchronize()
            xs = []
            for _ in range(args.amp_requests):
                t = time.perf_counter()
                net.run(amp=ampt, stream=side_stream)
                side_stream.synchronize()
                xs.append(1e3 * (time.perf_counter() - t))
            a_ = ampt.cpu().numpy()
            key = mode if not slice_sum else mode + "_slice_sum"
            lat[key] = {"p50_ms": percentile(xs, 50), "p99_ms": percentile(xs, 99),
                        "amplitudes_per_s": 1e3 / float(np.mean(xs)),
                        "amplitude": [float(a_[0]), float(a_[1])],
                        "flops_per_amplitude": fl}
        ctx.set_option("slice_sum", 0)
        from workloads import paths as _paths
        _, unsliced, _ = _paths.path_stats(w.network.labels, w.path)
        # Roofline of the batched-slice runs: each step at max(F / peak,
        # B / HBM), the steps back to back.
        for key in ("fp64", "fp32_4m"):
            es, peak = (16, FP64_PEAK) if key == "fp64" else (8, FP32_PEAK)
            F, B, T = network_roofline(w.network.labels, w.path, w.sliced, es, peak)
            lat[key].update({"model_flops": F, "model_bytes": B, "roofline_time_ms": 1e3 * T,
                             "roofline_frac_of_p50": 1e3 * T / lat[key]["p50_ms"]})
        if not args.no_cpu_baseline:
            t = time.perf_counter()
            ref_amp = complex(oracle.contract_network(w.network.tensors, w.network.labels,
                                                      w.path, w.sliced)[0])
            t_net = time.perf_counter() - t
            t = time.perf_counter()
            psi = oracle.statevector(w.circuit)
            t_sv = time.perf_counter() - t
            sv = complex(psi[int("".join(map(str, w.bitstring)), 2)])
            floor = 2.0 ** (-w.circuit.n / 2)
            for key, v in lat.items():
                a_ = complex(*v["amplitude"])
                v["e_amp_vs_oracle"] = abs(a_ - ref_amp) / max(abs(ref_amp), floor)
                v["e_amp_vs_statevector"] = abs(a_ - sv) / max(abs(sv), floor)
                v["tolerance"] = 1e-12 if key.startswith("fp64") else 1e-5
            lat["oracle"] = {"network_s": t_net, "statevector_s": t_sv,
                             "amplitude": [ref_amp.real, ref_amp.imag],
                             "statevector_amplitude": [sv.real, sv.imag],
                             "oracle_vs_statevector": abs(ref_amp - sv) / max(abs(sv), floor)}
        amp = {"workload": "one amplitude of a 20-qubit random circuit (4x5 grid, 12 cycles), "
                           "greedy path, 4 sliced bonds = 16 slices batched, FP64 slice sum; "
                           "one request at a time.  *_slice_sum: each sliced bond summed in "
                           "the step that contracts it (slices as blocks)", **lat,
               "flops": {"independent_slices": w.meta["flops_per_slice"] * (1 << len(w.sliced)),
                         "batched_broadcast": lat["fp64"]["flops_per_amplitude"],
                         "batched_broadcast_model": lat["fp64"]["model_flops"],
                         "slice_sum": lat["fp64_slice_sum"]["flops_per_amplitude"],
                         "unsliced_same_path": unsliced}}
        log(f"amplitude latency: {amp}")

        # Slices viewed as blocks on a circuit where slicing matters more:
        # 6x6 grid, 10 cycles, sliced until the largest intermediate has rank
        # <= 20 (6 bonds).  Independent slices redo every step per slice;
        # batching broadcasts what does not depend on a slice; slice-sum also
        # sums each sliced bond where it is contracted.
        w6 = configs.circuit_workload(6, 6, 10, 777, max_rank=20, restarts=2)
        ts = [torch.from_numpy(np.ascontiguousarray(t.reshape(-1))).to(torch.complex64).to(dev)
              for t in w6.network.tensors]
        sab = {"workload": "one amplitude, 36-qubit random circuit (6x6 grid, 10 cycles), "
                           f"{len(w6.sliced)} sliced bonds, FP32-4M",
               "flops": {"independent_slices": w6.meta["flops_per_slice"] << len(w6.sliced)}}
        vals = {}
        for name, ss in (("batched_broadcast", 0), ("slice_sum", 1)):
            ctx.set_option("slice_sum", ss)
            net = ctx.prepare_network(ts, w6.network.labels, w6.path, w6.sliced, "fp32_4m")
            ampt = torch.zeros(2, dtype=torch.float64, device=dev)
            xs = []
            for it in range(3 + 10):
                t = time.perf_counter()
                with torch.cuda.stream(side_stream):
                    net.run(amp=ampt)
                side_stream.synchronize()
                if it >= 3:
                    xs.append(1e3 * (time.perf_counter() - t))
            a_ = ampt.cpu().numpy()
            vals[name] = complex(a_[0], a_[1])
            sab["flops"][name] = net.flops
            sab[name] = {"p50_ms": percentile(xs, 50), "workspace_bytes": net.ws_bytes}
            del net
        ctx.set_option("slice_sum", 0)
        ref6 = vals["batched_broadcast"]
        sab["rel_diff_slice_sum_vs_batched"] = abs(vals["slice_sum"] - ref6) / max(
            abs(ref6), 2.0 ** (-w6.circuit.n / 2))
        amp["slices_as_blocks"] = sab
        log(f"slices as blocks: {sab}")

    # ------------------------------- uneven batch: 256 problems, one call
    batch = None
    if args.batch:
        t0 = time.time()
        probs = configs.config4()
        items = [(torch.from_numpy(p.a.data).to(torch.complex64).to(dev), p.a.dims, p.a.grid,
                  torch.from_numpy(p.b.data).to(torch.complex64).to(dev), p.b.dims, p.b.grid,
                  p.axes_a, p.axes_b) for p in probs]
        log(f"batch: 256 problems generated and uploaded in {time.time() - t0:.1f}s")
        # Descriptors, plan, outputs and workspace built once; each call then
        # only hashes the descriptors and replays the batch's HIP graph.
        pb = ctx.prepare_batch(items, "fp32_4m")
        pb.autotune()
        pb.run()
        bflops = pb.flops
        torch.cuda.synchronize()
        for _ in range(3):
            with torch.cuda.stream(side_stream):
                pb.run()
            side_stream.synchronize()
        reps = 20
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        t = time.perf_counter()
        with torch.cuda.stream(side_stream):
            ev0.record(side_stream)
            for _ in range(reps):
                pb.run()
            ev1.record(side_stream)
        side_stream.synchronize()
        el = (time.perf_counter() - t) / reps
        gpu_el = ev0.elapsed_time(ev1) / 1e3 / reps
        tstar = 0.0
        tbytes = 0.0
        for p in probs:
            m = 2 ** (len(p.a.dims) - p.k)
            n_ = 2 ** (len(p.b.dims) - p.k)
            kk = 2 ** p.k
            f_i = 8.0 * m * n_ * kk
            b_i = 8.0 * (m * kk + n_ * kk + m * n_)
            tbytes += b_i
            tstar += max(f_i / (FP32_PEAK * 1e12), b_i / (HBM_PEAK * 1e9))
        batch = {"workload": "256 independent block tensordots, operand ranks 8-24, 2-10 "
                             "contracted axes in random order, output rank <= 24, first three "
                             "axes of each operand split in two; complex64 FP32-4M; autotuned "
                             "tiles, grouped launches replayed as a HIP graph",
                 "ms": 1e3 * el, "gpu_ms_events": 1e3 * gpu_el, "tflops": bflops / el / 1e12,
                 "gbps_algorithmic": tbytes / el / 1e9,
                 "roofline_time_ms": 1e3 * tstar, "roofline_frac": tstar / el}
        log(f"batch: {batch}")
        del items, pb
        torch.cuda.empty_cache()

    # ------------------------------- serving: Poisson stream of requests
    serving = None
    if args.serve_requests > 0:
        serving, reqs = run_serving(args, torch, rn, log)
        if not args.no_cpu_baseline:
            serving["oracle_check"] = serving_oracle_sample(args, torch, rn, oracle, reqs, log)

    k = main_res["kernels"]
    gemm_ms = k["gemm"][0] / max(k["gemm"][1], 1)
    achieved = flops / (gemm_ms * 1e-3) / 1e12
    traffic = traffic_from_profiles("cgemm_f32_4m", 1)
    modes = {"fp32_4m": {"tflops": main_res["tflops"], "ms_per_step": main_res["ms_per_step"],
                         "errors_sampled": errors.get("fp32_4m"), "tolerance": 1e-5,
                         "frac_of_fp32_peak": main_res["tflops"] / FP32_PEAK}}
    for mode, r in side.items():
        modes[mode] = {"tflops": r["tflops"], "ms_per_step": r["ms_per_step"],
                       "errors_sampled": errors.get(mode),
                       "tolerance": {"fp64": 1e-12, "fp64_gauss": 1e-12,
                                     "fp32_3m": 1e-5}.get(mode, 1e-3)}
    if "fp64" in side:
        modes["fp64"]["frac_of_fp64_peak"] = side["fp64"]["tflops"] / FP64_PEAK
        modes["speedup_fp32_vs_fp64"] = main_res["tflops"] / side["fp64"]["tflops"]
    if "fp64_gauss" in side:
        modes["fp64_gauss"]["executed_frac_of_fp64_peak"] = (
            0.75 * side["fp64_gauss"]["tflops"] / FP64_PEAK)
    if "fp32_3m" in side:
        modes["fp32_3m"]["executed_frac_of_fp32_peak"] = 0.75 * side["fp32_3m"]["tflops"] / FP32_PEAK
    if "bf16x3_gauss" in side:
        modes["bf16x3_gauss"]["executed_frac_of_bf16_peak"] = (
            2.25 * side["bf16x3_gauss"]["tflops"] / BF16_PEAK)
    if "bf16x3" in side:
        modes["bf16x3"]["executed_frac_of_bf16_peak"] = 3 * side["bf16x3"]["tflops"] / BF16_PEAK
        if "fp64" in side:
            modes["speedup_bf16x3_vs_fp64"] = side["bf16x3"]["tflops"] / side["fp64"]["tflops"]

    line = {
        "metric": "block-tensordot TFLOP/s (FP64 vs FP32 vs split-BF16) + p50/p99 amplitude "
                  "latency",
        "value": main_res["tflops"],
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"pairwise contraction of two rank-{args.rank} complex64 tensors "
                               f"(all dims 2), {args.k} contracted indices in seeded random "
                               f"order, unblocked; FP32-4M; step = permute A, permute B, "
                               f"fused-pair complex GEMM, FP64 norm of C",
                   "M": M, "N": N, "K": K, "useful_flops_per_step": flops},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": FP32_PEAK,
                     "unit": "TFLOP/s", "frac": achieved / FP32_PEAK, "traffic": traffic,
                     "kernel": "FP32-4M complex GEMM (cgemm_f32_dl<1,4,4,1,16>, default large tile, direct-to-LDS staging)",
                     "kernel_ms": gemm_ms},
        "cpu_baseline": cpu,
        "modes": modes,
        "config1": config1,
        "amplitude_latency": amp,
        "batch": batch,
        "serving": serving,
        "kernel_ms_per_step": {kk: v[0] / args.steps for kk, v in k.items()},
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
