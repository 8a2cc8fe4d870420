"""Benchmark: 2D-OMP + TMOD signals/s per iteration on one MI355X.

One step = one iteration of Algorithm 1 (2D-OMP, D1 update, 2D-OMP, D2 update)
over all N signals of the workload, synthetic and already resident in HBM.  The
default workload is the image-patch-shaped FP32 problem: 8x8 signals, D1 and D2
8x16 (256 Kronecker atoms), s = 8, N = 100,000.

Prints ONE JSON line.  Also reports, for the dominant kernel (the 2D-OMP
sparse-coding kernel), its average device time measured with HIP events on the
stream it runs on, the algorithmic FLOP count per launch and the fraction of the
FP32 peak (157.3 TFLOP/s for both the vector units and the matrix cores); and the
FP64 CPU oracle timed on a bounded sample on this host's cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X FP32 vector (published)
HBM_PEAK_GBS = 8000.0


def omp_flops_per_signal(m1, m2, n1, n2, s):
    """Algorithmic FLOPs of one signal's 2D-OMP: first correlation D1^T Y D2 plus the
    Gram-form correlation refresh with t nonzeros at step t."""
    f_c = 2 * min(n1 * m2 * (m1 + n2), m1 * n2 * (m2 + n1))
    f_greedy = s * (s + 1) * n1 * n2
    return f_c + f_greedy


def sums_flops_per_signal(m1, m2, n1, n2, s):
    """Algorithmic FLOPs of one signal's contribution to one side's TMOD sums, using the
    sparsity of X_k: B += Y_k T_k^T touches only the s used atom columns (2 s m1 m2) and
    A += X_k G X_k^T has s^2 nonzero products (2 s^2)."""
    return 2 * s * m1 * m2 + 2 * s * s


def sums_flops_executed_per_signal(m1, m2, n1, n2, s):
    """FLOPs the sums epilogue actually executes per signal (dense T_k = X_k D2^T and dense
    products on the matrix cores, symmetric A in full), averaged over the two sides."""
    side1 = 2 * s * m2 + 2 * n1 * n1 * m2 + 2 * m1 * n1 * m2
    side2 = 2 * s * m1 + 2 * n2 * n2 * m1 + 2 * m2 * n2 * m1
    return (side1 + side2) / 2


def log(msg):
    """Progress line on stderr (the JSON result is the only line on stdout)."""
    print("bench: " + msg, file=sys.stderr, flush=True)


def median(v):
    v = sorted(v)
    return v[len(v) // 2]


def timed_runs(run, reps):
    """reps runs of run(), each bracketed by torch.cuda.synchronize() and by HIP events on the
    current stream; returns (median wall seconds, median event seconds, all wall seconds)."""
    import torch
    walls, evs = [], []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record()
        run()
        e1.record()
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        evs.append(e0.elapsed_time(e1) * 1e-3)
    return median(walls), median(evs), walls


def omp_bytes_per_signal(m1, m2, s, elem):
    # Y read once, supp (int32) + coef + res2 written
    return m1 * m2 * elem + s * (4 + elem) + elem


def kernel_symbol(w, tuned):
    """Name of the sparse-coding kernel instantiation the autotuner chose, as the
    profiler lists it."""
    if not tuned:
        return "omp_generic_kernel"
    lr, lc, wpe, mfma = tuned[:4]
    if mfma:
        return "omp_mfma_kernel<MCfg<%d, %d, %d, %d, %d, %d>>" % (w.m1, w.m2, w.n1, w.n2, w.s, wpe)
    return "omp_fast_kernel<Cfg<%d, %d, %d, %d, %d, %d, %d, %d>>" % (w.m1, w.m2, w.n1, w.n2, w.s, lr, lc, wpe)


def measured_traffic(w, symbol):
    """HBM bytes per launch of the sparse-coding kernel from the committed hardware-counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter reads for a copy of
    known size), or None when there is none for this kernel and workload or the kernel's
    sources have changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "omp_mfma_%s_traffic.json" % w.name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel") != symbol:
        return None
    h = hashlib.sha256()
    for src in t["sources"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    return t["bytes_per_launch"] if h.hexdigest() == t["source_sha256"] else None


def learned_vs_plain(args, api, oracle, synth):
    """Learned proposal + 2D-OMP fallback vs plain 2D-OMP, Algorithm 1 on 1M held-out signals
    of the learned workload (8x8, 16x16 atoms, s = 8), starting at the generating dictionaries;
    the network is trained on the 2D-OMP supports of 500k signals."""
    import torch

    w = synth.WORKLOADS["learned_8x8_n16_s8"]
    d1, d2 = synth.true_dictionaries(w)
    ntr, nev = 500_000, 1_000_000
    D1 = torch.from_numpy(d1.T.copy()).cuda()
    D2 = torch.from_numpy(d2.T.copy()).cuda()
    Ytr = torch.from_numpy(synth.signals(w, 0, ntr, dtype=np.float32, layout="colmajor")).cuda()
    tr = api.Problem(Ytr, D1.clone(), D2.clone(), w.s)
    api.sparse_code(tr)
    torch.cuda.synchronize()
    net = api.Proposer(w.m1, w.m2, w.n1, w.n2, hidden=512, seed=7)
    log("learned leg: training on %d signals" % ntr)
    t0 = time.perf_counter()
    losses = net.train(Ytr, tr.supp, w.s, epochs=8, batch=256, lr=1e-3)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    Yev = torch.from_numpy(synth.signals(w, ntr, ntr + nev, dtype=np.float32, layout="colmajor")).cuda()
    del Ytr, tr
    cal = api.Problem(Yev[:20000].contiguous(), D1.clone(), D2.clone(), w.s)
    tau = net.calibrate(cal)
    log("learned leg: calibrated, timing plain and learned Algorithm 1")
    st = api.new_stats()
    api.learned_sparse_code(net, api.Problem(Yev, D1.clone(), D2.clone(), w.s), tau=tau, stats=st)
    fallback_rate = st.fallbacks / nev
    K = args.learned_steps
    out = {"workload": w.name, "N": nev, "steps": K, "train_signals": ntr, "train_epochs": 8,
           "train_seconds": train_s, "final_train_loss": float(losses[-1]), "tau": tau,
           "fallback_rate": fallback_rate}
    nsub = 5000
    Ysub = synth.signals(w, ntr, ntr + nsub)
    for name, kw in (("plain", {}), ("learned", {"proposer": net, "tau": tau})):
        pr = api.Problem(Yev, D1.clone(), D2.clone(), w.s)

        def run():
            pr.D1.copy_(D1)
            pr.D2.copy_(D2)
            api.learn(pr, K, **kw)

        run()  # warm-up (captures the learning graph)
        dt, _, _ = timed_runs(run, 3)
        s_o, _, r_o = oracle.omp(Ysub, pr.d1(), pr.d2(), w.s, p=min(16, os.cpu_count() or 1))
        r_g = pr.res2[:nsub].double().cpu().numpy()
        out[name + "_value"] = nev * K / dt
        out[name + "_rmse_vs_oracle"] = float(np.sqrt(r_g.mean()) / np.sqrt(r_o.mean()))
        out[name + "_support_agreement"] = support_agreement(pr.supp[:nsub].cpu().numpy(), s_o)["support_agreement"]
    out["unit"] = "signals/s per iteration"
    out["learned_over_plain"] = out["learned_value"] / out["plain_value"]
    return out


def support_agreement(supp_gpu, supp_oracle):
    """Fraction of signals whose support set equals the oracle's, and fraction of the oracle's
    chosen atoms that the GPU also chose (empty slots are -1 on both sides)."""
    g = np.sort(np.asarray(supp_gpu, np.int64), axis=1)
    o = np.sort(np.asarray(supp_oracle, np.int64), axis=1)
    same = float(np.mean(np.all(g == o, axis=1)))
    hit = ((g[:, :, None] == o[:, None, :]) & (o[:, None, :] >= 0)).any(axis=1).sum()
    return {"support_agreement": same, "atom_agreement": float(hit / max(1, int((o >= 0).sum())))}


def device_signals(synth, w, dtype, k0=0, k1=None, chunk=100_000):
    """Signals k0..k1 of workload w, generated in chunks straight into a device tensor
    in the ABI layout (each signal column-major)."""
    import torch
    k1 = w.N if k1 is None else k1
    Y = torch.empty((k1 - k0, w.m2, w.m1), dtype=dtype, device="cuda")
    for c0 in range(k0, k1, chunk):
        c1 = min(k1, c0 + chunk)
        Y[c0 - k0:c1 - k0] = torch.from_numpy(synth.signals(w, c0, c1, layout="colmajor")).to("cuda", dtype)
    return Y


def timed_learn(api, fresh, K, reps=3, **opts):
    """Autotune, one untimed run of K iterations (it also captures the learning graph), then the
    median of reps timed runs of K graph-replayed iterations of Algorithm 1, each from the initial
    dictionaries on the same buffers; returns (problems, trace, seconds)."""
    import torch
    api.autotune(fresh(), reps=3)
    probs = fresh()
    plist = probs if isinstance(probs, list) else [probs]
    init = [(p.D1.clone(), p.D2.clone()) for p in plist]
    traces = []

    def run():
        for p, (a, b) in zip(plist, init):
            p.D1.copy_(a)
            p.D2.copy_(b)
        traces.append(api.learn(probs, K, **opts))

    run()
    dt, _, _ = timed_runs(run, reps)
    torch.cuda.synchronize()
    return probs, traces[-1], dt


def kernel_name(api, w):
    t = api.tuned_config(w.m1, w.m2, w.n1, w.n2, w.s)
    if t is None:
        return "generic (one wave per signal, all in LDS)"
    if t[3] == 2:
        if t[2] == 4:
            return "register-resident, 16 lanes per signal on 4x4x1 MFMA quadrants, 4 signals per wave"
        return "register-resident, one wave per signal, correlations in 16x16 MFMA tiles"
    return "register-resident lanes %dx%d, %d waves/SIMD%s" % (t[0], t[1], t[2], ", refresh on MFMA" if t[3] else "")


def mixed_workload(api, oracle, synth):
    """Mixed precision at its own shape: 1M signals of 12x12 stored in bfloat16, 24x24 atoms,
    s = 12, K = 10 iterations from the random initial dictionaries, with the correlations on the
    BF16 matrix cores (SDL_MIXED_BF16); the same workload with bfloat16 storage and FP32 arithmetic
    and with FP32 signals (the plain path) for the ratios."""
    import torch
    w = synth.WORKLOADS["mixed_12x12_n24_s12"]
    Y = device_signals(synth, w, torch.bfloat16)
    e1, e2 = synth.initial_dictionaries(w)
    nsub = 5000
    Ysub = Y[:nsub].double().cpu().numpy().transpose(0, 2, 1)  # the rounded signals, math layout

    def fresh():
        return api.Problem(Y, torch.from_numpy(e1.T.copy()).cuda(), torch.from_numpy(e2.T.copy()).cuda(), w.s)

    def quality(pr):
        s_o, _, r_o = oracle.omp(Ysub, pr.d1(), pr.d2(), w.s, p=min(16, os.cpu_count() or 1))
        r_g = pr.res2[:nsub].double().cpu().numpy()
        return {"rmse_vs_oracle": float(np.sqrt(r_g.mean()) / np.sqrt(r_o.mean())),
                **support_agreement(pr.supp[:nsub].cpu().numpy(), s_o)}

    pr, trace, dt = timed_learn(api, fresh, w.iters, mixed=True)
    st = api.new_stats()
    api.sparse_code(fresh(), mixed=True, stats=st)
    torch.cuda.synchronize()
    out = {"workload": w.name, "N": w.N, "steps": w.iters,
           "dtype": "bf16 signals, bf16 matrix-core correlations with f32 accumulation, f32 near-tie re-score "
                    "and Cholesky, f64 solves",
           "value": w.N * w.iters / dt, "unit": "signals/s per iteration", "ms_per_step": dt / w.iters * 1e3,
           "rmse_first": float(trace[0][0]), "rmse_final": float(trace[0][-1]), **quality(pr),
           "near_tie_rescored_steps_per_signal": st.near_tie_rescores / w.N,
           "near_tie_overflow_steps_per_signal": st.near_tie_overflows / w.N,
           "omp_kernel": "bf16 4x4x4 MFMA direct-form correlations, 16 signals per wave"}
    del pr
    # bfloat16 storage with FP32 arithmetic
    pb, trace_b, dtb = timed_learn(api, fresh, w.iters)
    out["bf16_storage_value"] = w.N * w.iters / dtb
    out["bf16_storage_rmse_vs_oracle"] = quality(pb)["rmse_vs_oracle"]
    out["bf16_storage_kernel"] = kernel_name(api, w)
    del pb
    Yf = device_signals(synth, w, torch.float32)

    def fresh32():
        return api.Problem(Yf, torch.from_numpy(e1.T.copy()).cuda(), torch.from_numpy(e2.T.copy()).cuda(), w.s)

    _, trace32, dt32 = timed_learn(api, fresh32, w.iters)
    out["fp32_value"] = w.N * w.iters / dt32
    out["fp32_rmse_final"] = float(trace32[0][-1])
    out["mixed_over_fp32"] = out["value"] / out["fp32_value"]
    return out


def error_driven_workload(api, oracle, synth):
    """Error-driven 2D-OMP (the stopping rule of the paper's denoising runs, Sec. IV) on the plain
    workload's 100,000 FP32 signals at their true dictionaries: eps = 1.15 sigma sqrt(m1 m2),
    err2 = eps^2, cap s = m1 m2 / 2, on the one-wave-per-signal kernel compiled for that cap; one
    sparse-coding launch timed with HIP events (mean of 5)."""
    import torch
    w = synth.WORKLOADS["fp32_8x8_n16_s8"]
    Y = device_signals(synth, w, torch.float32)
    d1, d2 = synth.true_dictionaries(w)
    m = w.m1 * w.m2
    s = m // 2
    err2 = float((1.15 * w.sigma() * np.sqrt(m)) ** 2)
    pr = api.Problem(Y, torch.from_numpy(d1.T.copy()).cuda(), torch.from_numpy(d2.T.copy()).cuda(), s)
    api.sparse_code(pr, err2=err2)
    st = api.new_stats()
    for _ in range(5):
        api.sparse_code(pr, err2=err2, timing=1, stats=st)
    torch.cuda.synchronize()
    d = st.as_dict()
    ms = d["kernel_ms"]["sparse_code"] / d["kernel_launches"]["sparse_code"]
    supp = pr.supp.cpu().numpy()
    nsub = 3000
    Ysub = Y[:nsub].double().cpu().numpy().transpose(0, 2, 1)
    s_o, _, _ = oracle.omp(Ysub, d1, d2, s, err2=err2, p=min(16, os.cpu_count() or 1))
    nbytes = w.N * (4 * m + 8 * s + 4)  # signals in; supp, coef, res2 out
    return {"workload": w.name + " with the error-driven stop", "N": w.N, "s_cap": s, "err2": err2,
            "value": w.N / ms * 1e3, "unit": "signals/s", "kernel_ms": ms,
            "mean_atoms": float((supp >= 0).sum(axis=1).mean()), "max_atoms": int((supp >= 0).sum(axis=1).max()),
            "hbm_gbs": nbytes / (ms * 1e-3) / 1e9,
            "omp_kernel": "omp_wave_mfma_kernel (one wave per signal, correlations in a 16x16 MFMA tile)",
            **support_agreement(supp[:nsub], s_o)}


def ortho_workload(api, oracle, synth):
    """Remark 1's orthonormal variant (hard-thresholded codes, orthogonal Procrustes updates) at the
    size of the paper's m = n = 8, s = 8 timing: 128,000 FP32 signals 8x8, K = 20 iterations from
    random orthonormal dictionaries; the sparse-coding launch timed with HIP events against its HBM
    bytes (signals in, codes out)."""
    import torch
    w = synth.WORKLOADS["ortho_8x8_s8"]
    Y = device_signals(synth, w, torch.float32)
    e1, e2 = synth.initial_dictionaries(w)

    def fresh():
        return api.Problem(Y, torch.from_numpy(e1.T.copy()).cuda(), torch.from_numpy(e2.T.copy()).cuda(), w.s)

    pr, trace, dt = timed_learn(api, fresh, w.iters, method=1)
    st = api.new_stats()
    p2 = fresh()
    for _ in range(5):
        api.sparse_code(p2, method=1, timing=1, stats=st)
    torch.cuda.synchronize()
    d = st.as_dict()
    ms = d["kernel_ms"]["sparse_code"] / d["kernel_launches"]["sparse_code"]
    nsub = 5000
    Ysub = synth.signals(w, 0, nsub)
    s_o, _, r_o = oracle.ortho_code(Ysub, pr.d1(), pr.d2(), w.s, p=min(16, os.cpu_count() or 1))
    r_g = pr.res2[:nsub].double().cpu().numpy()
    nbytes = w.N * (4 * w.m1 * w.m2 + 8 * w.s + 4)
    return {"workload": w.name, "N": w.N, "steps": w.iters, "value": w.N * w.iters / dt,
            "unit": "signals/s per iteration", "ms_per_step": dt / w.iters * 1e3,
            "rmse_first": float(trace[0][0]), "rmse_final": float(trace[0][-1]),
            "rmse_vs_oracle": float(np.sqrt(r_g.mean()) / np.sqrt(r_o.mean())),
            **support_agreement(pr.supp[:nsub].cpu().numpy(), s_o),
            "code_kernel_ms": ms, "code_hbm_gbs": nbytes / (ms * 1e-3) / 1e9,
            "code_kernel": "omp_mfma_kernel<MCfg<8, 8, 8, 8, 8, 3>, true> (first correlation on 4x4x1 MFMA, "
                           "exact top-s selection, Procrustes B sums in the epilogue)"}


def psnr(ref, img, peak=255.0):
    return float(10.0 * np.log10(peak * peak / np.mean((ref - img) ** 2)))


def denoise_workload(api, oracle, synth):
    """The denoising experiment of Sec. IV on a synthetic 512 x 512 image (FP32), sigma = 20:
    dictionaries learned from 4000 of its noisy 8 x 8 patches (s = 6, K = 20, from overcomplete-DCT
    starting dictionaries), 8 x 16 by Algorithm 1 and 8 x 8 orthonormal by the Remark 1 variant;
    then all 255,025 overlapping patches coded by the error-driven 2D-OMP (eps = 1.15 sigma
    sqrt(m1 m2), cap m1 m2 / 2) and the image rebuilt.  Timed: one whole denoising pass
    (extraction, coding, rebuild; median of 3)."""
    import torch
    H = W = 512
    sigma, s_train, K, n_train = 20.0, 6, 20, 4000
    clean = synth.synthetic_image(3, H, W)
    noisy = synth.noisy_image(clean, 3, sigma)
    img = torch.as_tensor(noisy, dtype=torch.float32, device="cuda")
    P = api.image_to_patches(img, 8, 8)
    idx = torch.as_tensor(synth.training_patch_index(3, P.shape[0], n_train), device="cuda")
    Ytr = P[idx].contiguous()
    err2 = float((1.15 * sigma) ** 2 * 64)
    rs = np.random.default_rng(0)
    ks = rs.choice(P.shape[0], 2000, replace=False)
    Pm = P[torch.as_tensor(ks, device="cuda")].double().cpu().numpy().transpose(0, 2, 1)
    out = {"image": "synthetic 512 x 512 (smooth background, rectangles, discs, stripes), FP32",
           "sigma": sigma, "patches": int(P.shape[0]), "train_patches": n_train, "train_s": s_train,
           "train_iters": K, "eps2": err2, "s_cap": 32, "psnr_noisy": psnr(clean, noisy)}
    for name, n, method in (("general_8x16", 16, 0), ("ortho_8x8", 8, 1)):
        d0 = synth.overcomplete_dct(8, n)
        D1 = torch.as_tensor(d0.T.copy(), device="cuda")
        D2 = D1.clone()
        pr = api.Problem(Ytr, D1, D2, s_train)
        if method == 0:
            api.autotune(pr, reps=1)
        tr = api.learn(pr, K, method=method)[0]
        st = api.new_stats()
        res = []

        def run():
            res.append(api.denoise(img, pr.D1, pr.D2, sigma, stats=st))

        run()
        dt, _, _ = timed_runs(run, 3)
        den, dp = res[-1]
        torch.cuda.synchronize()
        g = den.double().cpu().numpy()
        so, _, _ = oracle.omp(Pm, pr.d1(), pr.d2(), 32, err2=err2, p=min(16, os.cpu_count() or 1))
        sg = dp.supp[torch.as_tensor(ks, device="cuda")].cpu().numpy()
        out[name] = {"train_rmse_first": float(tr[0]), "train_rmse_final": float(tr[-1]),
                     "denoise_ms": dt * 1e3, "patches_per_s": P.shape[0] / dt,
                     "psnr": psnr(clean, g),
                     "mean_atoms": float((dp.supp >= 0).sum(dim=1).double().mean().item()),
                     "sampled_vs_oracle": support_agreement(sg, so)}
    return out


def tensor_workload(api, synth):
    """Remark 3's n-dimensional generalisation on a three-mode stand-in for hyperspectral patches:
    100,000 FP32 signals of 8 x 8 x 4, dictionaries 8 x 12, 8 x 12, 4 x 6 (864 atoms), s = 8,
    K = 10 iterations of Algorithm 1 with one sweep per mode (three sparse codings and three
    dictionary updates per iteration); plus one sparse-coding launch timed alone."""
    import torch
    from oracle import tensor as ot
    w = synth.TENSOR_WORKLOADS["tensor_8x8x4_n12x12x6_s8"]
    Y = synth.tensor_signals(w)
    E = synth.tensor_dictionaries(w, initial=True)
    pr = api.TensorProblem.from_math(Y, E, w.s, dtype=torch.float32)
    D0 = [d.clone() for d in pr.Ds]
    traces = []

    def run():
        for d, d0 in zip(pr.Ds, D0):
            d.copy_(d0)
        traces.append(api.tensor_learn(pr, w.iters))

    run()
    dt, _, _ = timed_runs(run, 3)
    pc = api.TensorProblem.from_math(Y, pr.dicts(), w.s, dtype=torch.float32)
    api.tensor_sparse_code(pc)
    _, code_s, _ = timed_runs(lambda: api.tensor_sparse_code(pc), 5)
    ms_, ns_ = w.ms, w.ns
    fc, pre, post = 0, 1, int(np.prod(ms_))
    for d in range(len(ms_)):
        post //= ms_[d]
        fc += 2 * pre * ns_[d] * ms_[d] * post
        pre *= ns_[d]
    A = int(np.prod(ns_))
    flops = w.N * (fc + w.s * (w.s + 1) * A)
    nsub = 500
    so, _, ro = ot.tensor_omp(Y[:nsub].astype(np.float32).astype(np.float64), pr.dicts(), w.s)
    rg = pc.res2[:nsub].double().cpu().numpy()
    return {"workload": w.name, "N": w.N, "modes": list(ms_), "atoms": list(ns_), "s": w.s, "steps": w.iters,
            "value": w.N * w.iters / dt, "unit": "signals/s per iteration (three sweeps and updates each)",
            "ms_per_step": dt / w.iters * 1e3, "rmse_first": float(traces[-1][0]),
            "rmse_final": float(traces[-1][-1]),
            "rmse_vs_oracle": float(np.sqrt(rg.mean()) / np.sqrt(ro.mean())),
            **support_agreement(pc.supp[:nsub].cpu().numpy(), so),
            "code_ms": code_s * 1e3, "code_tflops": flops / code_s / 1e12,
            "code_frac_fp32": flops / code_s / 1e12 / FP32_VECTOR_PEAK_TFLOPS,
            "code_kernel": "omp_wave_mfma_kernel<WCfg<8, 32, 12, 72, 8, ...>> (modes 2 and 3 collapsed into one "
                           "Kronecker factor: 8 x 32 signals, 12 x 72 atoms)",
            "sums_kernel": "tensor_sums_mfma_kernel<3> (16x16x4 FP32 MFMA over the concatenated W and Y)"}


def uneven_workload(api, oracle, synth):
    """The uneven batch: four problems of different shapes and sizes (370k signals in all)
    learned together in one call, K = 10."""
    import torch
    ws = [synth.WORKLOADS[n] for n in synth.UNEVEN_BATCH]
    Ys = [device_signals(synth, w, torch.float32) for w in ws]
    inits = [synth.initial_dictionaries(w) for w in ws]

    def fresh():
        return [api.Problem(Y, torch.from_numpy(e1.T.copy()).cuda(), torch.from_numpy(e2.T.copy()).cuda(), w.s)
                for Y, (e1, e2), w in zip(Ys, inits, ws)]

    K = ws[0].iters
    probs, trace, dt = timed_learn(api, fresh, K)
    ntot = sum(w.N for w in ws)
    per = []
    for w, pr, tr in zip(ws, probs, trace):
        nsub = 2000
        Ysub = synth.signals(w, 0, nsub)
        s_o, _, r_o = oracle.omp(Ysub, pr.d1(), pr.d2(), w.s, p=min(16, os.cpu_count() or 1))
        r_g = pr.res2[:nsub].double().cpu().numpy()
        per.append({"workload": w.name, "N": w.N, "rmse_final": float(tr[-1]),
                    "rmse_vs_oracle": float(np.sqrt(r_g.mean()) / np.sqrt(r_o.mean())),
                    **support_agreement(pr.supp[:nsub].cpu().numpy(), s_o),
                    "omp_kernel": kernel_name(api, w)})
    return {"N": ntot, "steps": K, "value": ntot * K / dt, "unit": "signals/s per iteration",
            "ms_per_step": dt / K * 1e3, "problems": per}


def cpu_baseline(args, oracle, synth, w, d1, d2):
    """The FP64 oracle (Algorithm 1, plain C loops) built with -O3 -march=native for this host, timed
    on a bounded prefix of the same workload: with as many threads as the process may use and with
    one thread; each one warm-up run and the median of three."""
    import tempfile
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    p = max(1, min(int(os.environ.get("OMP_NUM_THREADS", cores)), cores))
    with tempfile.TemporaryDirectory(prefix="sdlref_") as tmp:
        lib = oracle.build_native(tmp)
        out = {}
        for name, threads, ns, K in (("all", p, min(args.cpu_sample, w.N), args.cpu_iters),
                                     ("single", 1, min(args.cpu_sample_1t, w.N), args.cpu_iters_1t)):
            Yc = synth.signals(w, 0, ns)
            times = []
            for r in range(4):  # one warm-up, then three timed
                t0 = time.perf_counter()
                oracle.learn(Yc, d1, d2, w.s, K, p=threads, lib=lib)
                if r:
                    times.append(time.perf_counter() - t0)
            # K iterations (+ the final sparse coding the call includes) over ns signals
            out[name] = {"value": ns * K / median(times), "threads": threads, "signals": ns, "iterations": K,
                         "seconds_median": median(times)}
    a = out["all"]
    return {"value": a["value"], "unit": "signals/s per iteration", "cores": a["threads"], "kind": "oracle",
            "sample": "first %d signals of the workload, %d Algorithm-1 iterations plus the final 2D-OMP, FP64 "
                      "oracle built -O3 -march=native, %d threads, median of 3 after a warm-up"
                      % (a["signals"], a["iterations"], a["threads"]),
            "single_thread": {"value": out["single"]["value"], "unit": "signals/s per iteration", "cores": 1,
                              "sample": "first %d signals, %d iterations plus the final 2D-OMP, 1 thread, median "
                                        "of 3 after a warm-up" % (out["single"]["signals"],
                                                                   out["single"]["iterations"])},
            "seconds": {k: v["seconds_median"] for k, v in out.items()}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="fp32_8x8_n16_s8")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--runs", type=int, default=5, help="timed runs of K steps; the median is reported")
    ap.add_argument("--cpu-sample", type=int, default=100000)
    ap.add_argument("--cpu-iters", type=int, default=10)
    ap.add_argument("--cpu-sample-1t", type=int, default=10000)
    ap.add_argument("--cpu-iters-1t", type=int, default=5)
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--learned-steps", type=int, default=5)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-uneven", action="store_true")
    ap.add_argument("--no-error-driven", action="store_true")
    ap.add_argument("--no-ortho", action="store_true")
    ap.add_argument("--no-denoise", action="store_true")
    ap.add_argument("--no-tensor", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first run one elementwise FP32 copy of MIB MiB (reads and writes MIB MiB): "
                         "the reference dispatch that scales hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the TMOD sums would be all-reduced across GPUs; see the design notes).", file=sys.stderr)
        sys.exit(2)

    import torch

    import oracle
    from paper_2007_03800_amd import api, synth

    if args.copy_probe > 0:
        n = args.copy_probe * (1 << 20) // 4
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    w = synth.WORKLOADS[args.workload]
    dtype = torch.float32 if not args.workload.startswith("fp64") else torch.float64
    elem = 4 if dtype == torch.float32 else 8
    dev = "cuda"
    Yh = synth.signals(w, 0, w.N, dtype=np.float64, layout="colmajor")
    d1, d2 = synth.initial_dictionaries(w)
    Y = torch.from_numpy(Yh).to(device=dev, dtype=dtype).contiguous()
    del Yh

    def fresh():
        return api.Problem(Y, torch.from_numpy(d1.T.copy()).to(dev), torch.from_numpy(d2.T.copy()).to(dev), w.s)

    log("plain workload %s: autotune, warm-up, timed runs" % w.name)
    pr = fresh()
    # pick the sparse-coding kernel variant for this shape on this device (outside the timed region)
    if dtype == torch.float32:
        api.autotune(pr, reps=5)
    tuned = api.tuned_config(w.m1, w.m2, w.n1, w.n2, w.s) if dtype == torch.float32 else None
    if args.warmup > 0:
        api.learn(pr, args.warmup)
    torch.cuda.synchronize()
    # the timed problem keeps its buffers across runs (the library replays the learning graph it
    # captured for them); each run starts again from the initial dictionaries
    D1_0, D2_0 = pr.D1.clone(), pr.D2.clone()
    traces = []

    def run():
        pr.D1.copy_(D1_0)
        pr.D2.copy_(D2_0)
        traces.append(api.learn(pr, args.steps)[0])

    run()  # captures the graph for K = steps (not timed)
    elapsed, elapsed_ev, all_runs = timed_runs(run, args.runs)
    trace = traces[-1]
    value = w.N * args.steps / elapsed

    # dominant kernel timing: same workload, eager launches bracketed by HIP events on their stream
    st = api.new_stats()
    pr2 = fresh()
    api.learn(pr2, min(args.steps, 5), timing=1, stats=st)
    sd = st.as_dict()
    omp_ms = sd["kernel_ms"]["sparse_code"] / sd["kernel_launches"]["sparse_code"]
    # the launch codes every signal and accumulates its share of the next update's sums
    flops = (omp_flops_per_signal(w.m1, w.m2, w.n1, w.n2, w.s) +
             sums_flops_per_signal(w.m1, w.m2, w.n1, w.n2, w.s)) * w.N
    flops_exec = (omp_flops_per_signal(w.m1, w.m2, w.n1, w.n2, w.s) +
                  sums_flops_executed_per_signal(w.m1, w.m2, w.n1, w.n2, w.s)) * w.N
    achieved_tflops = flops / (omp_ms * 1e-3) / 1e12
    per_class = {k: round(v / sd["kernel_launches"][k], 4) for k, v in sd["kernel_ms"].items()}

    # matched RMSE: the oracle's 2D-OMP at the final GPU dictionaries on a 5000-signal prefix
    nsub = min(5000, w.N)
    Ysub = synth.signals(w, 0, nsub)
    s_o, _, r_o = oracle.omp(Ysub, pr.d1(), pr.d2(), w.s, p=min(16, os.cpu_count() or 1))
    r_g = pr.res2[:nsub].double().cpu().numpy()
    rmse_ratio = float(np.sqrt(r_g.mean()) / np.sqrt(r_o.mean()))
    agree = support_agreement(pr.supp[:nsub].cpu().numpy(), s_o)

    log("plain workload timed; kernel timing, oracle check")
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args, oracle, synth, w, d1, d2)

    # measured ceilings of this device (copy kernel, FMA and MFMA chains)
    log("measured ceilings")
    measured = {"hbm_copy_gbs": api.probe_hbm_copy(1 << 30, reps=5)}
    for k in api.PROBE_KINDS:
        measured[k + "_tflops"] = api.probe_peak(k, reps=5)
    peak_meas = measured["fp32_mfma_4x4x1_tflops" if tuned and tuned[3] else "fp32_fma_tflops"]

    log("learned proposal leg")
    learned = None
    if not args.no_learned and dtype == torch.float32:
        learned = learned_vs_plain(args, api, oracle, synth)
    log("mixed-precision leg")
    mixed = None if args.no_mixed else mixed_workload(api, oracle, synth)
    log("uneven-batch leg")
    uneven = None if args.no_uneven else uneven_workload(api, oracle, synth)
    log("error-driven leg")
    errdriven = None if args.no_error_driven else error_driven_workload(api, oracle, synth)
    log("orthonormal leg")
    ortho = None if args.no_ortho else ortho_workload(api, oracle, synth)
    log("denoising leg")
    denoise = None if args.no_denoise else denoise_workload(api, oracle, synth)
    log("n-dimensional leg")
    tensor = None if args.no_tensor else tensor_workload(api, synth)
    log("done")

    symbol = kernel_symbol(w, tuned)
    out = {
        "metric": "2D-OMP+TMOD signals/s per iteration, learned vs plain at matched RMSE",
        "value": value,
        "unit": "signals/s per iteration",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "timing": {"runs": args.runs, "statistic": "median", "wall_ms_per_step_runs":
                   [round(t / args.steps * 1e3, 5) for t in all_runs],
                   "event_ms_per_step": elapsed_ev / args.steps * 1e3},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if dtype == torch.float32 else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "path": "plain", "m1": w.m1, "m2": w.m2, "n1": w.n1, "n2": w.n2,
                   "s": w.s, "N": w.N, "snr_db": w.snr_db,
                   "omp_kernel": ("register-resident lanes %dx%d, %d waves/SIMD%s" %
                                  (tuned[0], tuned[1], tuned[2], ", refresh on MFMA" if tuned[3] else ""))
                   if tuned else "generic"},
        "roofline": {"bound": "mfma" if tuned and tuned[3] else "alu",
                     "kernel": symbol, "achieved": achieved_tflops,
                     "peak": FP32_VECTOR_PEAK_TFLOPS if elem == 4 else 78.6, "unit": "TFLOP/s",
                     "frac": achieved_tflops / (FP32_VECTOR_PEAK_TFLOPS if elem == 4 else 78.6),
                     "traffic": measured_traffic(w, symbol), "traffic_unit": "bytes/launch",
                     "avg_ms": omp_ms, "flops_per_launch": flops, "flops_executed_per_launch": flops_exec,
                     "frac_executed": flops_exec / (omp_ms * 1e-3) / 1e12 /
                     (FP32_VECTOR_PEAK_TFLOPS if elem == 4 else 78.6),
                     "peak_measured": peak_meas, "frac_measured": achieved_tflops / peak_meas},
        "measured_peaks": measured,
        "kernel_avg_ms": per_class,
        "rmse_final": float(trace[-1]),
        "rmse_vs_oracle": rmse_ratio,
        **agree,
        "learned_vs_plain": learned,
        "mixed_precision": mixed,
        "uneven_batch": uneven,
        "error_driven": errdriven,
        "orthonormal": ortho,
        "denoising": denoise,
        "tensor": tensor,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
