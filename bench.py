#!/usr/bin/env python3
"""Throughput of truncating an HT sum by the hierarchical SVD on one MI355X.

Workload (the paper's runtime tests use random H-tensors with n = 10 000 and
d up to 64): two seeded HT tensors with d = 64, n = 10 000, k = 64 (float32
N(0,1) leaf frames, transfer tensors with singular values 0.9^i), summed
lazily (sum rank 128) and truncated to relative accuracy 1e-6 by
ht_truncate: CholeskyQR2 orthogonalisation bottom-up, reduced Gramians
top-down, eigen-decompositions, rank selection and projection.  A "step" is
one such sum-truncation with all inputs resident in HBM.

Prints one JSON line (stdout).  The mixed-precision path is the headline
value; the float64 path and the fixed-rank (r = 64) reading are timed beside
it.  `roofline` describes the kernel with the largest share of the timed
region (HIP events around every launch, on the stream it runs on) and
`roofline_mfma` the matrix-core kernel with the largest share; `traffic` is
the committed rocprofv3 counter figure while the kernel sources match it.
`cpu_baseline` times the float64 NumPy oracle on one sum-truncation of the
same workload on the host cores.  `graph_ms_per_step` replays the headline step captured in a HIP graph.
`batched` times 256 uneven sums in one ht_truncate_batched call.
`inner_product` times <A, C> by Definition (phi) and the
difference norm ||A - C|| on the same inputs.  `large_single` times the large single
workload (d = 128, n = 1e5, k = 64 per summand, truncated to rank 64) and
ht_entries of its result at 1e6 random multi-indices.  `operator_apply`
times ht_apply (Lemma (operator)) at d = 64, n = 400, ranks 20, and `cg`
the steps of truncated CG (Algorithm (CG)) at d = 64, n = 1000.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAKS = {"double": 78.6e12, "float": 157.3e12}   # MI355X dense MFMA peaks, FP64 / FP32
HBM_PEAK = 8.0e12
FP64_VECTOR_PEAK = 78.6e12                           # MI355X float64 vector peak
ALU_KERNELS = ("eig_kernel", "chol_kernel")          # dense node solvers on the vector ALUs


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed(fn, steps, torch):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, reps=3):
    """Sum-truncations of the same workload by the float64 oracle: the median
    wall clock of `reps` runs (input generation excluded)."""
    import statistics
    from threadpoolctl import threadpool_info
    import htsynth as S
    from oracle import ht_oracle as O
    a, c = S.workload_pair("d64_n1e4_k64")
    A, C = O.from_input(a), O.from_input(c)
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        X = O.add(A, C)
        O.truncate(X, mode="tol", eps=cfg["eps"], relative=True)
        times.append(time.perf_counter() - t0)
        log(f"bench: oracle sum-truncation {times[-1]:.2f} s")
    dt = statistics.median(times)
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    return dict(value=1.0 / dt, unit="sum-truncations/s", cores=int(threads), kind="oracle",
                nproc=os.cpu_count(), cpu_model=cpu_model(), runs_s=[round(t, 3) for t in times],
                sample=f"median of {reps} full sum-truncations of the same workload (d=64, n=1e4, k=64+64, "
                       f"rel. tol {cfg['eps']:g}) by the float64 NumPy oracle, {dt:.1f} s each; "
                       f"cores = BLAS threads used")


def kernel_source_digest():
    """sha256 over the HIP sources and headers the kernels are built from."""
    import hashlib
    h = hashlib.sha256()
    cdir = os.path.join(ROOT, "paper_1708_03340_amd", "csrc")
    for name in sorted(os.listdir(cdir)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(cdir, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when there is none or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_d64_n1e4_k64.txt")
    if not os.path.exists(path):
        return None
    digest, rows = None, {}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line.startswith("source_sha256:"):
                digest = line.split(":", 1)[1].strip()
            elif line.startswith("kernel "):
                kv = dict(p.split("=", 1) for p in line.split()[1:])
                rows[kv["name"]] = float(kv["bytes_per_launch"])
    if digest != kernel_source_digest():
        return None
    return rows.get(kernel)


def device_tensor(H, torch, d, n, k, spectrum, gen):
    """One HT tensor of the large single workload, drawn on the device: float32
    N(0,1) leaf frames, transfer tensors with M_1(B_t) = P diag(g) W^T (P, W
    orthonormal from QR of N(0,1) matrices), float64 root of the same form."""
    tr = H.ht_tree(d)
    nn = 2 * d - 1
    g = torch.tensor(spectrum, dtype=torch.float64, device="cuda") if spectrum is not None else None

    def orth(rows, cols):
        q, _ = torch.linalg.qr(torch.randn(rows, cols, dtype=torch.float64, device="cuda", generator=gen))
        return q

    leaves, transfer, ranks = [None] * d, [None] * nn, [1] * nn
    for t in range(nn):
        if int(tr["son1"][t]) < 0:
            leaves[int(tr["lo"][t])] = torch.randn(k, n, dtype=torch.float32, device="cuda", generator=gen)
            ranks[t] = k
        elif spectrum is None:   # N(0,1) transfer tensors
            shape = (k, k) if t == 0 else (k, k, k)
            transfer[t] = torch.randn(*shape, dtype=torch.float64 if t == 0 else torch.float32, device="cuda",
                                      generator=gen)
            ranks[t] = 1 if t == 0 else k
        elif t == 0:
            transfer[t] = (orth(k, k) * g[None, :]) @ orth(k, k).T
        else:
            transfer[t] = ((orth(k, k) * g[None, :]) @ orth(k * k, k).T).reshape(k, k, k).float()
            ranks[t] = k
    return H.DeviceHT(d, [n] * d, ranks, leaves, transfer, 0)


def batched(H, torch, steps=3):
    """The batched workload: 256 independent sums A_b + C_b, d ~ U{4..32},
    n ~ U[100, 4096], k ~ U{8..48} (the same meta draw as the tests), N(0,1)
    float32 frames and transfer tensors drawn on the device, each truncated
    to its own k in the mixed path by one ht_truncate_batched call."""
    import htsynth as S
    meta = S.batched_meta()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(4)
    problems = []
    for m in meta:
        A = device_tensor(H, torch, m["d"], m["n"], m["k"], None, gen)
        C = device_tensor(H, torch, m["d"], m["n"], m["k"], None, gen)
        problems.append(dict(Xs=[A, C], mode=H.HT_RANK_FIXED, ranks=[m["k"]] * (2 * m["d"] - 1),
                             precision=H.HT_PREC_MIXED))
    bt = H.BatchTruncator(problems)
    bt()
    t = timed(bt, steps, torch)
    t_graph = graph_replay(H, torch, bt, steps)
    H.profile_enable(True)
    H.profile_reset()
    bt()
    torch.cuda.synchronize()
    prof = H.profile_read()
    H.profile_enable(False)
    H.profile_reset()
    flops = sum(e["flops"] for e in prof)
    launches = sum(e["launches"] for e in prof)
    log(f"bench: batched 256 sums {t * 1e3:.2f} ms per batch, {launches} launches, "
        f"{flops / t / 1e12:.2f} TF/s of algorithmic flops")
    out = dict(workload="256 HT sums in one ht_truncate_batched call: d ~ U{4..32}, n ~ U[100,4096], "
                        "k ~ U{8..48} per summand, each truncated to its own k (mixed precision)",
               ms_per_batch=t * 1e3, value=256.0 / t, unit="sum-truncations/s", steps=steps,
               graph_ms_per_batch=t_graph * 1e3,
               launches_per_batch=launches, alg_flops=flops, achieved_tflops=flops / t / 1e12,
               frac_fp64_peak=flops / t / PEAKS["double"])
    del problems, bt
    torch.cuda.empty_cache()
    return out


def graph_replay(H, torch, tr, steps):
    """The same call (a Truncator or BatchTruncator) captured once in a HIP
    graph and replayed."""
    tr()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        tr(stream=s)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            tr(stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g.replay()
    t = timed(g.replay, steps, torch)
    log(f"bench: graph replay {t * 1e3:.3f} ms/step")
    return t


def large_single(H, torch, steps=3):
    """The large single workload: d=128, n=1e5, k=64 per summand, spectra
    10^(-i/16), the sum truncated to rank 64 (mixed path), then ht_entries of
    the result at 1e6 random multi-indices."""
    d, n, k, m = 128, 100000, 64, 1000000
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    spec = [10.0 ** (-i / 16.0) for i in range(k)]
    log("bench: large single workload d=128 n=1e5 k=64+64 -> 64 (inputs drawn on the device)")
    A, C = device_tensor(H, torch, d, n, k, spec, gen), device_tensor(H, torch, d, n, k, spec, gen)
    tr = H.Truncator([A, C], [1.0, 1.0], mode=H.HT_RANK_FIXED, ranks=[k] * (2 * d - 1), precision=H.HT_PREC_MIXED)
    res = tr()
    t_trunc = timed(tr, steps, torch)
    log(f"bench: large single {t_trunc * 1e3:.2f} ms per sum-truncation")
    idx = torch.randint(0, n, (m, d), dtype=torch.int32, device="cuda", generator=gen)
    H.ht_entries(res.out, idx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H.ht_entries(res.out, idx)
    torch.cuda.synchronize()
    t_ent = time.perf_counter() - t0
    log(f"bench: large single ht_entries {m} indices in {t_ent * 1e3:.1f} ms")
    out = dict(workload="HT sum truncation d=128 n=100000 k=64+64 -> 64 (mixed precision), then entries at 1e6 "
                        "random multi-indices", ms_per_step=t_trunc * 1e3, value=1.0 / t_trunc,
               unit="sum-truncations/s", steps=steps, entries_m=m, entries_ms=t_ent * 1e3, entries_per_s=m / t_ent)
    del A, C, tr, res, idx
    torch.cuda.empty_cache()
    return out


def inner_products(H, torch, A, C, a, c, steps=20, with_cpu=True):
    """<A, C> by Definition (phi) and the difference norm ||A - C|| (lazy sum
    orthogonalised, root norm) on the d=64 workload; achieved float64 rate
    from the launches' algorithmic flops; the oracle's <A, C> timed beside it."""
    phi = H.Inner(A, C)
    dn = H.Norm([A, C], [1.0, -1.0])

    phi(); dn()
    t_phi = timed(phi, steps, torch)
    t_dn = timed(dn, steps, torch)
    H.profile_enable(True)
    H.profile_reset()
    phi()
    torch.cuda.synchronize()
    prof = H.profile_read()
    H.profile_enable(False)
    H.profile_reset()
    flops = sum(e["flops"] for e in prof)
    kern_ms = sum(e["ms"] for e in prof)
    out = dict(workload="<A, C> by Definition (phi), d=64 n=10000 k=64 (float32 frames), and ||A - C|| "
                        "by orthogonalising the lazy difference",
               inner_ms=t_phi * 1e3, inner_per_s=1.0 / t_phi, diff_norm_ms=t_dn * 1e3,
               inner_alg_flops=flops, inner_achieved_tflops=flops / t_phi / 1e12,
               inner_frac_fp64_peak=flops / t_phi / PEAKS["double"], inner_kernel_ms=kern_ms)
    log(f"bench: <A,C> {t_phi * 1e3:.3f} ms ({flops / t_phi / 1e12:.2f} TF/s of algorithmic flops), "
        f"||A - C|| {t_dn * 1e3:.3f} ms")
    if with_cpu:
        from oracle import ht_oracle as O
        Ao, Co = O.from_input(a), O.from_input(c)
        t0 = time.perf_counter()
        O.inner(Ao, Co)
        out["cpu_oracle_inner_s"] = time.perf_counter() - t0
        log(f"bench: oracle <A,C> {out['cpu_oracle_inner_s']:.2f} s")
    return out


def operator_apply(H, torch, steps=5):
    """Lemma (operator) at the paper's operator workload: d = 64, n = 400,
    tensor and operator ranks 20 (the product has ranks 400), N(0,1) float32
    frames and transfer tensors drawn on the device, output preallocated.
    The Kronecker kernel writes every product transfer tensor (400^3 float32
    per inner node) and is bound by HBM writes."""
    d, n, k = 64, 400, 20
    nn = 2 * d - 1
    gen = torch.Generator(device="cuda")
    gen.manual_seed(400)
    L = device_tensor(H, torch, d, n * n, k, None, gen)
    A = device_tensor(H, torch, d, n, k, None, gen)
    C = H.DeviceHT.empty(d, [n] * d, [1] + [k * k] * (nn - 1), torch.float32, torch.float32)
    H.ht_apply(L, A, C)
    t = timed(lambda: H.ht_apply(L, A, C), steps, torch)
    H.profile_enable(True)
    H.profile_reset()
    H.ht_apply(L, A, C)
    torch.cuda.synchronize()
    prof = H.profile_read()
    H.profile_enable(False)
    H.profile_reset()
    kron = [e for e in prof if e["kernel"].startswith("kron_kernel")]
    kms = sum(e["ms"] for e in kron)
    kbytes = sum(e["bytes"] for e in kron)
    out = dict(workload="H-operator application (Lemma (operator)) d=64 n=400, operator and tensor ranks 20 "
                        "(product ranks 400), float32",
               ms_per_apply=t * 1e3, value=1.0 / t, unit="operator applications/s", steps=steps,
               kron_ms=kms, kron_alg_bytes=kbytes,
               kron_roofline=dict(bound="hbm", achieved=kbytes / (kms * 1e-3) / 1e9 if kms else None,
                                  peak=HBM_PEAK / 1e9, unit="GB/s",
                                  frac=kbytes / (kms * 1e-3) / HBM_PEAK if kms else None))
    log(f"bench: operator application {t * 1e3:.3f} ms; Kronecker kernel {kms:.3f} ms, "
        f"{kbytes / max(kms * 1e-3, 1e-12) / 1e9:.0f} GB/s")
    del L, A, C
    torch.cuda.empty_cache()
    return out


def cg_solver(H, torch, steps=4):
    """Algorithm (CG) in HT arithmetic on the device: d = 64, n = 1000, the
    Kronecker-sum operator of M_mu = Q diag(U[1, 3]) Q^T / d (SPD, spectrum
    in [1, 3]), a right-hand side of ranks 8 (N(0,1) float64), T = fixed rank
    32 (float64 path).  One CG step is an operator application, four
    truncations of sums of rank 64 and two inner products; the figure is
    (time of `steps` steps - time of the start alone) / steps."""
    from paper_1708_03340_amd import solvers as SV
    d, n, kb = 64, 1000, 8
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1000)
    mats = []
    for _ in range(d):
        q, _ = torch.linalg.qr(torch.randn(n, n, dtype=torch.float64, device="cuda", generator=gen))
        lam = 1.0 + 2.0 * torch.rand(n, dtype=torch.float64, device="cuda", generator=gen)
        mats.append((q * lam[None, :]) @ q.T / d)
    Aop = SV.kron_sum_operator(mats)
    B = device_tensor(H, torch, d, n, kb, None, gen)
    B = H.DeviceHT(d, B.n, B.ranks, [u.double() for u in B.leaves],
                   [b.double() if b is not None else None for b in B.transfer], 0)
    T = SV.Trunc("fixed", rank=32)
    SV.cg(Aop, B, T, eps=0.0, max_steps=1)
    t0 = timed(lambda: SV.cg(Aop, B, T, eps=0.0, max_steps=0), 2, torch)
    hist = []
    tn = timed(lambda: SV.cg(Aop, B, T, eps=0.0, max_steps=steps, history=hist), 1, torch)
    per = (tn - t0) / steps
    out = dict(workload="truncated CG (Algorithm (CG)) d=64 n=1000, Kronecker-sum SPD operator, right-hand side "
                        "ranks 8, T = fixed rank 32 (float64)",
               ms_per_cg_step=per * 1e3, value=1.0 / per, unit="CG steps/s", steps=steps,
               residual_log2_norms=[0.5 * h["rr_log2"] for h in hist])
    log(f"bench: CG {per * 1e3:.2f} ms per step; log2 of the residual norms "
        + " ".join(f"{r:.1f}" for r in out["residual_log2_norms"]))
    del Aop, B, mats
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--fp64-steps", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the large single workload (d=128, n=1e5), the batch and the operator application")
    ap.add_argument("--no-cg", action="store_true", help="skip the truncated-CG figure")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline steps: no graph replay, inner products, batch, large, operator or CG "
                         "figures (for counter runs that divide by the number of steps)")
    ap.add_argument("--breakdown", action="store_true", help="print the per-step profile to stderr")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="before the benchmark, run three plain device copies of MIB MiB (a known "
                         "HBM traffic of 2*MIB MiB each) to scale hardware byte counters")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the truncation of one HT sum runs on one GPU and "
              "there is no multi-GPU path; use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1708_03340_amd as H
    import htsynth as S

    cfg = dict(d=64, n=10000, k=64, eps=1e-6)
    torch.cuda.set_device(0)
    if args.copy_calibration > 0:
        nel = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"bench: copy calibration, 3 copies of {args.copy_calibration} MiB")
        del src, dst
    log("bench: generating inputs (d=64, n=1e4, k=64, float32)")
    a, c = S.workload_pair("d64_n1e4_k64")
    A, C = H.DeviceHT.from_input(a), H.DeviceHT.from_input(c)
    torch.cuda.synchronize()
    mixed = H.Truncator([A, C], [1.0, 1.0], mode=H.HT_RANK_TOL, eps=cfg["eps"], relative=True,
                        precision=H.HT_PREC_MIXED)
    fp64 = H.Truncator([A, C], [1.0, 1.0], mode=H.HT_RANK_TOL, eps=cfg["eps"], relative=True,
                       precision=H.HT_PREC_FP64, out_frame_dtype=torch.float32, out_transfer_dtype=torch.float32)
    fixed = H.Truncator([A, C], [1.0, 1.0], mode=H.HT_RANK_FIXED, ranks=[64] * (2 * cfg["d"] - 1),
                        precision=H.HT_PREC_MIXED)

    log(f"bench: warmup {args.warmup}")
    for _ in range(args.warmup):
        res = mixed()
    torch.cuda.synchronize()
    ranks = res.ranks[1:]
    log(f"bench: ranks chosen min {min(ranks)} max {max(ranks)} flags {res.flags & 255} "
        f"max QL iterations {res.flags >> 8}")

    # timed region: K mixed-precision sum-truncations (the headline value)
    log(f"bench: timing {args.steps} steps (mixed)")
    t_mixed = timed(mixed, args.steps, torch)
    log(f"bench: mixed {t_mixed * 1e3:.3f} ms/step")
    # the same K steps again with HIP events around every launch, on the stream
    # each launch runs on: per-kernel durations for the roofline (the events
    # themselves cost a few percent, so the value above is timed without them)
    H.profile_enable(True)
    H.profile_reset()
    t_prof = timed(mixed, args.steps, torch)
    prof = H.profile_read()
    H.profile_enable(False)
    H.profile_reset()
    log(f"bench: mixed with launch events {t_prof * 1e3:.3f} ms/step")

    t_fp64 = t_fixed = None
    if args.fp64_steps > 0:
        for _ in range(2):
            fp64()
        t_fp64 = timed(fp64, args.fp64_steps, torch)
        log(f"bench: fp64 {t_fp64 * 1e3:.3f} ms/step")
        for _ in range(2):
            fixed()
        t_fixed = timed(fixed, args.fp64_steps, torch)
        log(f"bench: fixed r=64 (mixed) {t_fixed * 1e3:.3f} ms/step")

    # accuracy of the mixed path against the float64 path (outside the timed
    # region): both results evaluated by ht_entries at the same seeded random
    # multi-indices; relative 2-norm of the difference over the sample
    err_mixed = None
    if args.fp64_steps > 0:
        idx = torch.from_numpy(S.entry_indices(200000, cfg["d"], cfg["n"], seed=77)).cuda()
        vm = H.ht_entries(mixed().out, idx)
        vf = H.ht_entries(fp64().out, idx)
        torch.cuda.synchronize()
        err_mixed = float(torch.linalg.vector_norm(vm - vf) / torch.linalg.vector_norm(vf))
        log(f"bench: mixed vs float64 relative difference over 2e5 sampled entries {err_mixed:.3e}")

    # dominant kernel of the timed region (largest summed launch time)
    by_kernel = {}
    for e in prof:
        k = by_kernel.setdefault(e["kernel"], dict(ms=0.0, flops=0.0, bytes=0.0, launches=0, labels=set()))
        k["ms"] += e["ms"]; k["flops"] += e["flops"]; k["bytes"] += e["bytes"]; k["launches"] += e["launches"]
        k["labels"].add(e["label"])
    total_ms = sum(v["ms"] for v in by_kernel.values())

    def math_type(kname):
        # math type of a GEMM kernel: third template argument of gemm_kernel<A,B,math,acc64>
        # and gemm_rk_kernel<A,B,math,mode,kc,km>; gemm128_kernel and the streamed kernels
        # (gemm_sb_kernel, gemm_sb_ring_kernel) compute in float64
        if kname.startswith("gemm128_kernel") or kname.startswith("gemm_sb"):
            return "double"
        if kname.startswith("gemm_kernel") or kname.startswith("gemm_rk_kernel"):
            return kname[kname.index("<") + 1:].rstrip(">").split(",")[2]
        return None

    def roofline(kname, kd):
        common = dict(kernel=kname, avg_launch_us=kd["ms"] * 1e3 / kd["launches"],
                      launches_per_step=kd["launches"] / args.steps,
                      share_of_launch_time=kd["ms"] / total_ms,
                      profiled_ms_per_step=t_prof * 1e3,
                      alg_bytes_per_launch=kd["bytes"] / kd["launches"],
                      alg_flops_per_launch=kd["flops"] / kd["launches"])
        mt = math_type(kname)
        if mt in PEAKS:
            achieved = kd["flops"] / (kd["ms"] * 1e-3)
            return dict(bound="mfma", achieved=achieved / 1e12, peak=PEAKS[mt] / 1e12, unit="TFLOP/s",
                        frac=achieved / PEAKS[mt], traffic=measured_traffic(kname), **common)
        if kname.split("<")[0] in ALU_KERNELS:
            # latency-bound float64 vector code (one node per workgroup): priced
            # against the float64 vector peak
            achieved = kd["flops"] / (kd["ms"] * 1e-3)
            return dict(bound="alu", achieved=achieved / 1e12, peak=FP64_VECTOR_PEAK / 1e12, unit="TFLOP/s",
                        frac=achieved / FP64_VECTOR_PEAK, traffic=measured_traffic(kname), **common)
        achieved = kd["bytes"] / (kd["ms"] * 1e-3)
        return dict(bound="hbm", achieved=achieved / 1e9, peak=HBM_PEAK / 1e9, unit="GB/s",
                    frac=achieved / HBM_PEAK, traffic=measured_traffic(kname), **common)

    kname, kd = max(by_kernel.items(), key=lambda kv: kv[1]["ms"])
    roof = roofline(kname, kd)
    mfma_kernels = [kv for kv in by_kernel.items() if math_type(kv[0]) in PEAKS]
    roof_mfma = roofline(*max(mfma_kernels, key=lambda kv: kv[1]["ms"])) if mfma_kernels else None
    if args.breakdown or True:
        labels = {}
        for e in prof:
            l = labels.setdefault(e["label"], [0.0, 0.0, 0])
            l[0] += e["ms"]; l[1] += e["flops"]; l[2] += e["launches"]
        log("bench: per-step breakdown (ms per sum-truncation, achieved TFLOP/s):")
        for lab, (ms, fl, n) in sorted(labels.items(), key=lambda kv: -kv[1][0]):
            log(f"  {lab:22s} {ms / args.steps:8.3f} ms  {fl / max(ms * 1e-3, 1e-12) / 1e12:7.2f} TF/s  "
                f"{n / args.steps:5.1f} launches")
        log(f"  (sum of launch times {total_ms / args.steps:.3f} ms of {t_prof * 1e3:.3f} ms wall with events)")

    out = {
        "metric": "HT sum-truncations/s at d=64,n=1e4,k=64; mixed vs FP64 at rel err <=1e-6",
        "value": 1.0 / t_mixed,
        "unit": "sum-truncations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_mixed * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic (seeded; float32 N(0,1) leaf frames, transfer tensors with singular values 0.9^i)",
        "config": {"workload": "HT sum truncation d=64 n=10000 k=64+64 -> rel tol 1e-6 (mixed path: float32 inputs "
                               "and outputs; at this shape every product runs in float64, see speedup_mixed_vs_fp64)",
                   "d": 64, "n": 10000, "k": 64, "sum_rank": 128, "eps": cfg["eps"], "rank_rule": "tolerance",
                   "parallelism": "single GPU"},
        "fp64_value": 1.0 / t_fp64 if t_fp64 else None,
        "fp64_ms_per_step": t_fp64 * 1e3 if t_fp64 else None,
        "speedup_mixed_vs_fp64": t_fp64 / t_mixed if t_fp64 else None,
        "fixed_r64_value": 1.0 / t_fixed if t_fixed else None,
        "rel_err_mixed_vs_fp64": err_mixed,
        "rel_err_sample": "relative 2-norm difference of the two results over 2e5 seeded random entries",
        "ranks_chosen": [min(ranks), max(ranks)],
        "roofline": roof,
        "roofline_mfma": roof_mfma,
    }
    ex = not args.no_extras
    out["graph_ms_per_step"] = graph_replay(H, torch, mixed, args.steps) * 1e3 if ex else None
    out["inner_product"] = inner_products(H, torch, A, C, a, c, with_cpu=not args.no_cpu) if ex else None
    out["batched"] = None if (args.no_large or not ex) else batched(H, torch)
    out["large_single"] = None if (args.no_large or not ex) else large_single(H, torch)
    out["operator_apply"] = None if (args.no_large or not ex) else operator_apply(H, torch)
    out["cg"] = None if (args.no_cg or not ex) else cg_solver(H, torch)
    if not args.no_cpu:
        log("bench: CPU oracle baseline (one sum-truncation)")
        out["cpu_baseline"] = cpu_baseline(cfg)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
