#!/usr/bin/env python3
"""Throughput of encrypted quadratic-gradient NAG training on one MI355X.

Workload: the paper's full-batch experiment shape (section 5.1, Table 1):
422,108 synthetic samples x 200 features (+ bias, padded to 256 columns),
packed 128 rows per ciphertext into 3,298 CKKS ciphertexts, N = 2^16,
24 RNS limbs (60/40-bit), dnum = 4 hybrid key switching, scale 2^40,
degree-3 sigmoid g8.  One step = one encrypted QG-NAG iteration over every
block (steps 4-6 of section 4.3) plus the refresh of W and V (step 7, here
the key-holder refresh).  Inputs are resident in HBM before timing starts.

Prints one JSON line (metric, value in seconds per iteration, the NTT
row-pass roofline measured live with sampled HIP events, and the CPU oracle
timed on a bounded sample of the same workload).
"""
import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-instructions per second (a wave64
# instruction takes 4 cycles of a SIMD, FP64 and 32-bit integer operations alike)
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
# the bootstrap whose output level the iteration works at: EvalMod with r = 5 double angles and a
# degree-20 Taylor cosine (|I| < 16 with a weight-64 sparse secret), slot transforms factored into 2
# levels each (the dense form needs N/2 plaintexts per transform)
BOOT_R, BOOT_LEVELS, BOOT_TAYLOR, BOOT_WEIGHT = 5, 2, 20, 64
# the non-interactive pipeline (every iteration followed by bootstrapping W and V) on a chain of 50-bit
# primes, where bootstrapping is precise: 4 double angles, 3 levels per slot transform
NI_Q_BITS, NI_P_BITS, NI_LOG2_SCALE, NI_R, NI_LEVELS = [60] + [50] * 24, 60, 50, 4, 3
# FP64 vector issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz instructions per second (the published
# 78.6 TFLOP/s counts each FMA as two flops)
FP64_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
PMC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_c3.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2406_13221_amd", "csrc", "ntt.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(cfg, data, n_blocks, work=None):
    """The oracle timed on a bounded sample of the same iteration: the whole iteration (per-block
    pipeline and the once-per-iteration tail) over 1 and over 9 blocks; the difference gives the
    per-block cost, the rest is the tail; the iteration over all blocks is extrapolated from both.
    Z and B-bar sit at the top level, W and V at `work` (default: the top), as on the GPU."""
    import numpy as np
    from oracle import circuit, trainer
    from oracle.ckks import Oracle
    from oracle.encode import encode
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    o = Oracle.from_config(cfg)
    m, g = cfg["m"], cfg["g"]
    o.keygen(cfg["key_seed"], circuit.rot_steps(m, g))
    lo, hi = 1, 9
    X, y = data["X"][:hi * m], data["y"][:hi * m]
    blocks = circuit.pack_blocks(trainer.build_Z(X, y, g), m, g, o.N)
    from paper_2406_13221_amd.train import SIGMOID_SCALE
    L = o.top_level
    work = L if work is None else work
    Zc = [o.encrypt(encode(blocks[b], o.N, o.delta), L, o.delta, cfg["enc_seed"], b) for b in range(hi)]
    B = trainer.bbar(X, g)
    sB = 2.0 ** (cfg["log2_scale"] + 10) / B.max()
    Bc = o.encrypt(encode(circuit.replicate_row(B, m, g), o.N, sB), L, sB, cfg["enc_seed"], 10)
    W = o.encrypt(np.zeros(o.N, np.int64), work, o.delta, cfg["enc_seed"], 11)
    V = o.encrypt(np.zeros(o.N, np.int64), work, o.delta, cfg["enc_seed"], 12)
    masks = circuit.make_masks(o, m, g, trainer.G8, work, SIGMOID_SCALE)
    times = {}
    for nb in (lo, hi):
        t0 = time.perf_counter()
        circuit.nag_qg_step(o, Zc[:nb], Bc, W, V, circuit.new_state(refresh_seed=7), masks, m, g, degree=3)
        times[nb] = time.perf_counter() - t0
    per_block = (times[hi] - times[lo]) / (hi - lo)
    tail = max(times[lo] - lo * per_block, 0.0)
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), None)
    except OSError:
        pass
    return dict(value=tail + per_block * n_blocks, unit="s/iter", cores=threads, kind="oracle", cpu_model=model,
                sample="the full iteration (per-block pipeline + once-per-iteration tail) over %d and over %d "
                       "of the %d blocks at the same parameters and levels (W and V at level %d): %.1f s and %.1f s, "
                       "i.e. %.2f s per block and %.2f s for the tail, extrapolated to %d blocks"
                       % (lo, hi, n_blocks, work, times[lo], times[hi], per_block, tail, n_blocks))


def iteration_model_bytes(cfg, n_blocks, degree=3, level=None):
    """Bytes of one full-batch iteration if every primitive reads its inputs and writes its
    outputs once (a limb = 8N bytes; an NTT reads and writes each limb once; switching keys
    read once per iteration, so not counted per block), starting at `level` (default: the top)."""
    N, nq, np_, dnum = 1 << cfg["log2N"], len(cfg["q_bits"]), cfg["n_p"], cfg["dnum"]
    alpha = -(-nq // dnum)
    g, m = cfg["g"], cfg["m"]
    lg, lm = g.bit_length() - 1, m.bit_length() - 1

    def ks(n):                     # key switch of one part with n limbs (result: 2 parts)
        digits = [min(alpha, n - j * alpha) for j in range(-(-n // alpha))]
        ext = n + np_
        tgt = sum(ext - d for d in digits)
        return (2 * n                      # INTT of the input part
                + n + tgt                  # ModUp: read digits, write targets
                + 2 * tgt                  # NTT of the targets
                + len(digits) * ext + 2 * ext   # inner product: read extended digits, write 2 parts
                + 2 * 2 * np_              # INTT of the special rows
                + 2 * np_ + 2 * n          # ModDown conversion
                + 2 * 2 * n                # NTT of the conversion
                + 3 * 2 * n)               # (acc - conv) P^-1 + base: read 2, write 1

    def rescale(n, parts):         # n limbs -> n-1
        return parts * (2 + 2 * (n - 1) + 2 * n)   # INTT of the last limb, NTT of its spread, combine

    def hmult_rs(n):               # tensor + relin + rescale
        return 7 * n + ks(n) + 3 * 2 * n + rescale(n, 2)

    def add_rot(n):                # x + Rot(x)
        return ks(n) + 2 * n + 3 * 2 * n

    L = nq - 1 if level is None else level
    per_block = 0
    n = L + 1
    per_block += hmult_rs(n)                       # u = Z (x) W
    n -= 1
    per_block += lg * add_rot(n)                   # row sums
    per_block += 2 * (4 * n + rescale(n, 2))       # two masked plaintext products
    per_block += hmult_rs(n)                       # u^2
    n -= 1
    per_block += hmult_rs(n)                       # b3 * u^2
    if degree >= 5:
        per_block += hmult_rs(n)
    n -= 1
    per_block += 2 * 3 * n + 3 * n                 # additions, + F/2
    per_block += lg * add_rot(n)                   # replication
    per_block += 7 * n + 3 * 2 * n                 # Z (x) p accumulated
    tail = 3 * n + ks(n) + rescale(n, 2) + lm * add_rot(n - 1) + 2 * hmult_rs(n - 1)
    return 8.0 * N * (per_block * n_blocks + tail)


def pmc_traffic(kernel, batch, level, rows=None):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 --pmc summary (FETCH_SIZE and
    WRITE_SIZE per dispatch, scaled by what the counters read for a plain device copy, one entry
    per chunk size): for the conversion pass bytes per output row x `rows`, for the others bytes
    per dispatch.  None when the summary is missing, the NTT source has changed since it was
    taken, or it holds no entry for this chunk size or working level."""
    try:
        with open(PMC_FILE) as f:
            pm = json.load(f)
        with open(KERNEL_SRC, "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != pm["kernel_source_sha256"]:
                return None
        if pm["work_level"] != level or str(batch) not in pm["by_batch"]:
            return None
        k = pm["by_batch"][str(batch)]["kernels"][kernel]
        if rows is not None:
            return k["bytes_per_output_row"] * rows
        return k["fetch_bytes_per_dispatch"] + k["write_bytes_per_dispatch"]
    except (OSError, KeyError, ValueError, TypeError):
        return None


def pmc_valu(kernel, batch, level, launch_us):
    """VALU issue rate of `kernel`: its wave-level VALU instructions per dispatch from the committed
    rocprofv3 SQ summary (SQ_INSTS_VALU), times 64 lanes, over the launch duration measured in this
    run, against VALU_PEAK_LANE_OPS.  None under the same conditions as pmc_traffic, or where no SQ
    pass was taken at this chunk size."""
    try:
        with open(PMC_FILE) as f:
            pm = json.load(f)
        with open(KERNEL_SRC, "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != pm["kernel_source_sha256"]:
                return None
        if pm["work_level"] != level or str(batch) not in pm["by_batch"] or launch_us <= 0:
            return None
        insts = pm["by_batch"][str(batch)]["sq"][kernel]["valu_insts_per_dispatch"]
        rate = insts * 64 / (launch_us * 1e-6)
        return {"valu_insts_per_launch": round(insts), "lane_ops_per_s": rate, "peak_lane_ops_per_s": VALU_PEAK_LANE_OPS,
                "frac": round(rate / VALU_PEAK_LANE_OPS, 4)}
    except (OSError, KeyError, ValueError, TypeError):
        return None


def auroc(score, y):
    """Area under the ROC curve as the rank statistic (ties at mid-rank)."""
    from scipy.stats import rankdata
    r = rankdata(score)
    npos = int(y.sum())
    return float((r[y == 1].sum() - npos * (npos + 1) / 2.0) / (npos * (len(y) - npos)))


def loglik_auroc(Xv, yv, w):
    """Mean log-likelihood (section 2.3) and AUROC of the decrypted model w (bias first) on validation rows."""
    import numpy as np
    score = w[0] + Xv @ w[1:Xv.shape[1] + 1]
    ypm = 2.0 * yv - 1.0
    ll = -float(np.mean(np.logaddexp(0.0, -ypm * score)))
    return ll, auroc(score, yv)


def scoring_leg(run, cfg, data, level=2, sample_blocks=64):
    """Encrypted validation scoring: the client encrypts the validation rows [1 | X | 0] (no labels) at
    `level` (one product and the row-sum rotations need no more), the cloud computes every row's score
    x-hat . w under the encrypted model (heqg_score); timed over all rows; a sample of row blocks is
    decrypted and compared with the plaintext scores of the decrypted model."""
    import numpy as np
    import torch
    from paper_2406_13221_amd import heqg
    from paper_2406_13221_amd.train import pack_grid
    ctx, keys, m, g = run.ctx, run.keys, run.m, run.g
    Xv, yv = data["Xv"], data["yv"]
    n, f = Xv.shape
    Xh = np.zeros((n, run.width))
    Xh[:, 0] = 1.0
    Xh[:, 1:f + 1] = Xv
    blocks = pack_grid(Xh, m, g)
    nb = blocks.shape[0]
    t0 = time.perf_counter()
    cts = heqg.Cts(torch.empty((nb, 2, level + 1, ctx.N), dtype=torch.int64, device="cuda"), level, ctx.delta)
    ws = heqg._ws(heqg.lib().heqg_enc_ws_bytes(ctx.h, 256))
    for b0 in range(0, nb, 256):
        b1 = min(nb, b0 + 256)
        dev = torch.from_numpy(ctx.encode_batch(blocks[b0:b1], ctx.delta)).cuda()
        ob = heqg.Cts(cts.data[b0:b1], level, ctx.delta).batch()
        heqg._check(heqg.lib().heqg_encrypt(ctx.h, keys.handle, dev.data_ptr(), cfg["enc_seed"] + 300, b0,
                                            ctypes.byref(ob), ws.data_ptr(), ws.numel(), heqg._stream()))
    del ws
    torch.cuda.synchronize()
    t_enc = time.perf_counter() - t0
    W2 = ctx.drop(run.W, level)
    ctx.score(keys, heqg.Cts(cts.data[:run.batch * run.nc], level, ctx.delta), W2, g, col_blocks=run.nc,
              batch=run.batch, ws=run.ws)     # warm-up on one chunk
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sc = ctx.score(keys, cts, W2, g, col_blocks=run.nc, batch=run.batch, ws=run.ws)
    torch.cuda.synchronize()
    t_score = time.perf_counter() - t0
    w = run.weights(f + 1)
    nsb = min(sample_blocks, sc.count)
    got = np.concatenate([ctx.decrypt_values(keys, sc, index=i).reshape(m, g)[:, 0] for i in range(nsb)])
    rows = min(n, nsb * m)
    ref = Xh[:rows, :f + 1] @ w
    res = {"rows": n, "row_blocks": sc.count, "ciphertexts_in": int(cts.count), "level": level,
           "encrypt_s": round(t_enc, 3), "score_s": round(t_score, 4),
           "rows_per_s": round(n / t_score, 1), "sample_rows": rows,
           "sample_max_abs_err": float(np.abs(got[:rows] - ref).max()),
           "sample_auroc_encrypted": round(auroc(got[:rows], yv[:rows]), 6),
           "sample_auroc_plain": round(auroc(ref, yv[:rows]), 6)}
    del cts, sc
    torch.cuda.empty_cache()
    return res


def mnist_leg(steps, batch):
    import torch
    import synth
    from paper_2406_13221_amd.train import EncryptedQGNAG
    cfg = synth.get_config("c6")
    d = synth.make_dataset(cfg)
    g16 = {1: 0.0843, 3: -0.0002}   # least-squares cubic on [-16, 16] (section 4.1)
    res = {"workload": cfg["name"], "n_samples": cfg["n_train"], "n_features": cfg["n_features"],
           "n_valid": cfg["n_valid"], "rows_per_block": cfg["m"], "cols": cfg["g"], "sigmoid": "g16",
           "iterations": steps}
    for name, fo in (("quadratic_gradient", False), ("first_order_nag", True)):
        run = EncryptedQGNAG(cfg, d["X"], d["y"], coeffs=g16, batch=min(batch, 12), first_order=fo)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            run.step()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        w = run.weights(cfg["n_features"] + 1)
        ll_tr, _ = loglik_auroc(d["X"], d["y"], w)
        ll_v, auc = loglik_auroc(d["Xv"], d["yv"], w)
        res[name] = {"s_per_iter": round(dt, 4), "train_loglik": round(ll_tr, 5), "valid_loglik": round(ll_v, 5),
                     "valid_auroc": round(auc, 5)}
        log("mnist-shaped %s: %.3f s/iter, train loglik %.4f, valid AUROC %.4f" % (name, dt, ll_tr, auc))
        del run
        torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3")
    ap.add_argument("--batch", type=int, default=16, help="blocks per lock-step chunk")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--prof-every", type=int, default=16)
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (NTT split/variants, chunk size)")
    ap.add_argument("--graph-steps", type=int, default=1, help="timed graph-replayed full-batch iterations")
    ap.add_argument("--mini-steps", type=int, default=10, help="timed mini-batch steps (eager and graph)")
    ap.add_argument("--learned-steps", type=int, default=1,
                    help="0: skip the learned degree-5 and degree-7 forms (fitted, timed beside g8, and each trained "
                         "10 iterations on the 1,024 x 32 layout)")
    ap.add_argument("--grid-steps", type=int, default=1,
                    help="timed iterations of the same task over 1,024 x 32 blocks (7 column blocks, section 2.2)")
    ap.add_argument("--mnist-steps", type=int, default=3,
                    help="iterations of the MNIST-shaped task (section 5.2), quadratic gradient and first-order NAG")
    ap.add_argument("--no-score", dest="score", action="store_false",
                    help="skip encrypted scoring of the validation rows")
    ap.add_argument("--mode", default="train", choices=["train", "ntt"],
                    help="ntt: only the batched forward NTT (768 limbs) and a 1 GiB device copy, for counters")
    ap.add_argument("--work-level", default="boot",
                    help="level of W and V, the level they are refreshed to: 'boot' (the level heqg_bootstrap "
                         "returns with 5 double angles), 'top', or a number")
    ap.add_argument("--noninteractive-steps", type=int, default=3,
                    help="iterations of the non-interactive pipeline (iteration + bootstrapping of W and V) on "
                         "the chain of 50-bit primes (0: skip)")
    ap.add_argument("--boot-reps", type=int, default=2,
                    help="timed bootstraps of W and V at these parameters (0: skip)")
    ap.add_argument("--top-steps", type=int, default=1,
                    help="timed iterations with W and V at the top level")
    ap.add_argument("--paper-q-steps", type=int, default=0,
                    help="timed iterations at the paper's working modulus (Table 1: Q = 2^275)")
    ap.add_argument("--no-ntt-probe", dest="ntt_probe", action="store_false",
                    help="skip the full-batch NTT throughput leg (keeps per-kernel profiles to the iteration)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="end with a 1 GiB device copy (the scale of HBM byte counters in a profiled run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path (see DESIGN.md for how "
              "the iteration would shard by row blocks)", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_2406_13221_amd import heqg
    from paper_2406_13221_amd.train import EncryptedQGNAG

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    cfg = synth.get_config(args.config)
    if args.mode == "ntt":
        ctx = heqg.Context.from_config(cfg)
        rows = torch.randint(0, 2 ** 39, (16 * 2, ctx.n_q, ctx.N), dtype=torch.int64, device="cuda")
        for _ in range(3):
            ctx.ntt(rows, 0, ctx.n_q)
        src = torch.ones(1 << 27, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "ntt", "ntt_rows_per_launch": rows.shape[0] * rows.shape[1],
                          "copy_bytes": src.numel() * 8}), flush=True)
        return
    data = synth.make_dataset(cfg)
    t0 = time.perf_counter()
    run = EncryptedQGNAG(cfg, data["X"], data["y"], batch=args.batch)
    top = run.ctx.top_level
    work = {"top": top, "boot": run.ctx.boot_shape(BOOT_R, BOOT_LEVELS)[2]}.get(args.work_level)
    work = int(args.work_level) if work is None else work
    if work != top:
        run.reset(obj=(1 << 40) + 1, level=work)
    torch.cuda.synchronize()
    log("setup %.1f s, %d blocks, %.1f GB resident; Z at level %d, W and V at level %d" %
        (time.perf_counter() - t0, run.Z.count, torch.cuda.memory_allocated() / 1e9, top, work))
    tuning = None
    if not args.no_tune:
        tuning = run.tune()
        log("tuned: %s" % tuning)
    for i in range(args.warmup):
        run.step()
        torch.cuda.synchronize()
        log("warmup step %d done" % i)

    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    heqg.prof_start(args.prof_every)
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record()
        run.step(refresh=False)
        ev[k][1].record()
        depth_g8 = run.L - run.W.level
        run.refresh()
        ev[k][2].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    conv_us, conv_n, conv_rows, conv_src, conv_ops = heqg.prof_stop(1)
    avg_us, n_sampled, avg_rows, _, _ = heqg.prof_stop(0)
    ks_us, ks_n, ks_rows, ks_keyrows, _ = heqg.prof_stop(2)
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    upd = sum(e[0].elapsed_time(e[1]) for e in ev) / args.steps / 1000.0
    ref = sum(e[1].elapsed_time(e[2]) for e in ev) / args.steps / 1000.0
    log("timed %d steps: %.3f s/step (update %.3f s, refresh %.4f s)" % (args.steps, ms_per_step / 1e3, upd, ref))
    # the model after these iterations (g8 only so far), for the comparison with the 1,024 x 32 layout
    w_cmp, t_cmp = run.weights(cfg["n_features"] + 1), int(run.state.t)
    batch_used = run.batch
    # the data owner's FP64 run of the same iterations (the decrypted weights must follow it within 1e-3)
    w_fp64 = {t: heqg.plain_qgnag(data["X"], data["y"], t, coeffs=dict(run.coeffs), margins=False)[0]
              for t in (1, t_cmp)}
    fp64_check = {"iterations": t_cmp, "max_abs_dw": float(abs(w_cmp - w_fp64[t_cmp]).max())}
    log("decrypted weights after %d iterations: max|dw| vs FP64 %.2e" % (t_cmp, fp64_check["max_abs_dw"]))

    # the same iteration submitted as a replayed HIP graph (first call captures, untimed)
    graph_s = None
    if args.graph_steps > 0:
        run.graph, run.stream = True, torch.cuda.Stream()
        run.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.graph_steps):
            run.step()
        torch.cuda.synchronize()
        graph_s = (time.perf_counter() - t0) / args.graph_steps
        run.graph, run.stream = False, None
        run.ctx.graph_clear()
        log("graph-replayed iteration: %.3f s" % graph_s)

    # the learned-sigmoid form: odd degree-5 and degree-7 polynomials in m/8, fitted by FP32 Adam on the
    # GPU to sigma on the margins of the data owner's FP64 plaintext run with the exact sigmoid (10
    # iterations x 422,108 rows); here their cost per iteration on this layout (levels consumed, time),
    # their training quality below on the 1,024 x 32 layout (the same model, 10x cheaper iterations)
    learned, forms = None, None
    if args.learned_steps > 0:
        import numpy as np
        from paper_2406_13221_amd import sigmoid_fit
        t0 = time.perf_counter()
        _, margins = heqg.plain_qgnag(data["X"], data["y"], 10)
        t_traj = time.perf_counter() - t0
        forms = {"g8": dict(run.coeffs)}
        fit_info = {}
        for deg in (5, 7):
            t0 = time.perf_counter()
            c, trace = sigmoid_fit.fit(margins, deg, steps=2000)
            forms["degree%d" % deg] = sigmoid_fit.power_coeffs(c)
            fit_info["degree%d" % deg] = {"coeffs_of_m_over_8": [float(v) for v in c],
                                          "fit_s": round(time.perf_counter() - t0, 3), "final_mse": float(trace[-1])}
        g8 = dict(run.coeffs)
        learned = {"margins": int(margins.size), "trajectory_s": round(t_traj, 2), "fits": fit_info,
                   "layout_128x256": {}}
        for name, co in forms.items():
            run.set_sigmoid(co)
            run.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run.step(refresh=False)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            levels = run.L - run.W.level
            learned["layout_128x256"][name] = {"s_per_iter": round(dt, 4), "levels_per_iteration": levels}
            run.refresh()
            log("%s on 128 x 256: %.3f s/iter, %d levels" % (name, dt, levels))
        run.set_sigmoid(g8)

    # mini-batch steps (Algorithm 1, 1,024 rows = 8 blocks per batch), eager and graph-replayed
    mini = None
    if args.mini_steps > 0 and cfg.get("batch_rows"):
        import copy
        mb = run.with_batches(cfg["batch_rows"], batch=8)
        mb.step()
        torch.cuda.synchronize()
        st0 = copy.copy(mb.state)
        t0 = time.perf_counter()
        for _ in range(args.mini_steps):
            mb.step()
        torch.cuda.synchronize()
        eager_ms = (time.perf_counter() - t0) * 1e3 / args.mini_steps
        mb.graph, mb.stream = True, torch.cuda.Stream()
        mb.state = copy.copy(st0)
        for _ in range(args.mini_steps):     # capture one graph per batch
            mb.step()
        torch.cuda.synchronize()
        mb.state = copy.copy(st0)
        t0 = time.perf_counter()
        for _ in range(args.mini_steps):     # replay them
            mb.step()
        torch.cuda.synchronize()
        graph_ms = (time.perf_counter() - t0) * 1e3 / args.mini_steps
        run.ctx.graph_clear()
        mini = {"ms_per_step_eager": round(eager_ms, 2), "ms_per_step_graph": round(graph_ms, 2),
                "blocks_per_step": mb.block_spans[0][1] - mb.block_spans[0][0], "steps": args.mini_steps,
                "n_batches": len(mb.block_spans)}
        log("mini-batch step: eager %.2f ms, graph %.2f ms" % (eager_ms, graph_ms))
        del mb

    # NTT throughput over the full batch of the iteration: every limb of every part of the 3,298 Z
    # ciphertexts (3,298 x 2 x 24 rows, 40- and 60-bit primes, 83 GB: far past the caches), transformed
    # in place forward and then back, which restores Z exactly; bytes = read once + written once per limb
    N = run.ctx.N
    ntt_gbps = None
    if args.ntt_probe:
        zrows = run.Z.data.view(-1, N)
        nrows = zrows.shape[0]
        for _ in range(1):
            run.ctx.ntt(zrows, 0, run.ctx.n_q)
            run.ctx.ntt(zrows, 0, run.ctx.n_q, inverse=True)
        e0, e1, e2 = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        reps = 2
        e0.record()
        for _ in range(reps):
            run.ctx.ntt(zrows, 0, run.ctx.n_q)
            run.ctx.ntt(zrows, 0, run.ctx.n_q, inverse=True)
        e1.record()
        torch.cuda.synchronize()
        e1b, e2 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e1b.record()
        for _ in range(reps):
            run.ctx.ntt(zrows, 0, run.ctx.n_q)
        e2.record()
        torch.cuda.synchronize()
        for _ in range(reps):
            run.ctx.ntt(zrows, 0, run.ctx.n_q, inverse=True)
        torch.cuda.synchronize()
        ntt_bytes = 16.0 * N * nrows
        fwd_s = e1b.elapsed_time(e2) * 1e-3 / reps
        both_s = e0.elapsed_time(e1) * 1e-3 / reps
        fwd_gbs = ntt_bytes / fwd_s / 1e9
        inv_gbs = ntt_bytes / max(both_s - fwd_s, 1e-9) / 1e9
        ntt_gbps = {"forward": round(fwd_gbs, 1), "inverse": round(inv_gbs, 1), "limbs_per_call": nrows,
                    "bytes_per_call": ntt_bytes, "frac_of_hbm_peak": round(fwd_gbs / HBM_PEAK_GBS, 4),
                    "batch": "every limb of the iteration's ciphertexts (blocks x 2 parts x limbs), in place"}

    w = run.weights(cfg["n_features"] + 1)
    n_blocks = run.Z.count
    if not (abs(w).max() < 1e3):
        print("decrypted weights out of range", file=sys.stderr)
        sys.exit(1)

    # the base conversion (on the int8 matrix cores) fused into the first forward column pass.  Its algorithmic bytes: every output row written once, every distinct source row
    # read once; the roofline is those bytes per launch against the HBM peak, with the FP64 issue
    # figures beside it (the digit combine and the butterflies; the matrix products are a few percent
    # of the int8 peak)
    conv_bytes = 8.0 * N * (conv_rows + conv_src)
    conv_gbs = conv_bytes / (conv_us * 1e-6) / 1e9 if conv_us > 0 else 0.0
    conv_tops = conv_ops / (conv_us * 1e-6) / 1e12 if conv_us > 0 else 0.0
    conv_roofline = {"bound": "hbm", "achieved": round(conv_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(conv_gbs / HBM_PEAK_GBS, 4), "traffic": pmc_traffic("k_conv_cols", run.batch, work, rows=conv_rows),
                "kernel": "k_conv_cols<8,*> (ModUp / ModDown base conversion on the int8 matrix cores, fused "
                          "into the first forward NTT pass)",
                "bytes": "8 bytes per output residue written + 8 per source residue read, once",
                "algorithmic_bytes_per_launch": conv_bytes, "algorithmic_fp64_ops_per_launch": conv_ops,
                "fp64_ops": "output residues x (12 to combine the digit sums + 4 per stage)",
                "fp64_achieved_Tops": round(conv_tops, 2), "fp64_frac": round(conv_tops / FP64_PEAK_TOPS, 4),
                "avg_launch_us": round(conv_us, 2), "sampled_launches": conv_n,
                "avg_rows_per_launch": round(conv_rows, 2), "avg_source_rows_per_launch": round(conv_src, 2),
                "valu": pmc_valu("k_conv_cols", run.batch, work, conv_us)}
    row_pass = 16.0 * N * avg_rows / (avg_us * 1e-6) / 1e9 if avg_us > 0 else 0.0
    ntt_row_roofline = {"bound": "hbm", "achieved": round(row_pass, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(row_pass / HBM_PEAK_GBS, 4),
                        "kernel": "k_ntt_rows<8,true,*,false> (plain forward NTT, second pass)",
                        "avg_launch_us": round(avg_us, 2), "sampled_launches": n_sampled,
                        "avg_rows_per_launch": round(avg_rows, 2)}

    # dominant kernel: the ModUp row pass fused with the key inner product.  Its algorithmic bytes:
    # ciphertext rows read and written plus the switching-key rows, each read once per launch.  Its
    # HBM traffic per launch comes from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary, valid
    # for the chunk size and working level it was taken at
    ks_bytes = 8.0 * N * (ks_rows + ks_keyrows)
    ks_rate = ks_bytes / (ks_us * 1e-6) / 1e9 if ks_us > 0 else 0.0
    roofline = {"bound": "hbm", "achieved": round(ks_rate, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ks_rate / HBM_PEAK_GBS, 4), "traffic": pmc_traffic("k_ntt_rows_ks8", run.batch, work),
                "kernel": "k_ntt_rows_ks8 (ModUp second forward pass of every digit fused with the key inner "
                          "product; the P limbs' first inverse pass)",
                "bytes": "8 bytes per ciphertext residue read (digits) and written (2 parts), key rows once",
                "algorithmic_bytes_per_launch": ks_bytes, "avg_launch_us": round(ks_us, 2),
                "sampled_launches": ks_n, "valu": pmc_valu("k_ntt_rows_ks8", run.batch, work, ks_us)}

    model = iteration_model_bytes(cfg, run.Z.count, level=work)
    it_roof = {"model_bytes": model, "achieved_GBps": round(model / upd / 1e9, 1), "peak": HBM_PEAK_GBS,
               "frac": round(model / upd / 1e9 / HBM_PEAK_GBS, 4),
               "note": "each primitive reads its inputs and writes its outputs once; keys read once per iteration"}

    out = {
        "metric": "sec per encrypted QG-NAG iteration (422k x 200, N=2^16)",
        "value": round(ms_per_step / 1000.0, 4),
        "unit": "s/iter",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic (seeded; shapes of the paper's 422,108 x 200 workload)",
        "config": {"workload": "%s full-batch QG-NAG iteration + W/V refresh (Z at level %d, W and V at level %d)"
                               % (cfg["name"], top, work),
                   "n_samples": cfg["n_train"], "n_features": cfg["n_features"], "log2N": cfg["log2N"],
                   "limbs": len(cfg["q_bits"]), "dnum": cfg["dnum"], "blocks": run.Z.count,
                   "z_level": top, "work_level": work, "work_log2_modulus": int(sum(cfg["q_bits"][:work + 1])),
                   "rows_per_block": cfg["m"], "cols": cfg["g"], "batch_blocks": run.batch},
        "fp64_check": fp64_check,
        "update_s": round(upd, 4),
        "refresh_s": round(ref, 5),
        "ntt_gbps": ntt_gbps,
        "roofline": roofline,
        "conv_pass_roofline": conv_roofline,
        "ntt_row_pass_roofline": ntt_row_roofline,
        "iteration_roofline": it_roof,
        "graph_s_per_iter": None if graph_s is None else round(graph_s, 4),
        "minibatch": mini,
        "learned_sigmoid": learned,
        "tuning": tuning,
    }
    # encrypted validation scoring (844,217 rows) with the trained model
    scoring = None
    if args.score:
        scoring = scoring_leg(run, cfg, data)
        log("encrypted scoring of %d validation rows: %.3f s; sample AUROC %.5f (plain %.5f)" %
            (scoring["rows"], scoring["score_s"], scoring["sample_auroc_encrypted"], scoring["sample_auroc_plain"]))
    out["validation_scoring"] = scoring

    # CKKS bootstrapping at these parameters, the refresh the paper runs once per iteration (Table 1):
    # a key set on a sparse secret (weight 64) with the factored transforms' rotations and the
    # conjugation; W and V of the run above, decrypted and encrypted again at level 0 under it, are
    # bootstrapped together; time per bootstrap of the pair and the error of the decrypted result
    boot_leg = None
    if args.boot_reps > 0:
        import numpy as np
        ctx = run.ctx
        t0 = time.perf_counter()
        kb = ctx.keygen(cfg["key_seed"] + 1, ctx.boot_steps(BOOT_LEVELS), hamming=BOOT_WEIGHT, conj=True)
        torch.cuda.synchronize()
        t_keys = time.perf_counter() - t0
        t0 = time.perf_counter()
        pts = ctx.boot_encode(BOOT_R, BOOT_LEVELS)
        t_enc = time.perf_counter() - t0
        t0 = time.perf_counter()
        bt = ctx.boot_setup(pts, BOOT_R, BOOT_TAYLOR, levels=BOOT_LEVELS)
        t_setup = time.perf_counter() - t0
        del pts
        zs = [ctx.decrypt_values(run.keys, c) for c in (run.W, run.V)]
        ct = ctx.encrypt(kb, np.stack([ctx.encode(z, ctx.delta) for z in zs]), 0, ctx.delta, cfg["enc_seed"] + 11,
                         1 << 43)
        ws = heqg._ws(heqg.lib().heqg_boot_ws_bytes(ctx.h, BOOT_LEVELS, ct.count))
        out_b = ctx.bootstrap(kb, bt, ct, ws=ws)      # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.boot_reps):
            out_b = ctx.bootstrap(kb, bt, ct, ws=ws)
        torch.cuda.synchronize()
        t_boot = (time.perf_counter() - t0) / args.boot_reps
        err = max(float(np.abs(ctx.decrypt_values(kb, out_b, index=i) - zs[i]).max()) for i in range(2))
        cl, sl, ol, npts = ctx.boot_shape(BOOT_R, BOOT_LEVELS)
        boot_leg = {"ciphertexts": 2, "s_per_bootstrap": round(t_boot, 4), "levels_per_transform": BOOT_LEVELS,
                    "double_angles": BOOT_R, "taylor_degree": BOOT_TAYLOR, "secret_weight": BOOT_WEIGHT,
                    "input_level": 0, "output_level": ol, "rotation_keys": len(kb.galois), "plaintexts": npts,
                    "keygen_s": round(t_keys, 3), "encode_s": round(t_enc, 3), "setup_s": round(t_setup, 3),
                    "max_abs_err": err,
                    "note": "real bootstrapping of W and V; at a 40-bit scale with q0 = 2^60, EvalMod's error "
                            "is scaled up by q0 / (2 pi Delta) = 2^17.3, so the result is not usable as a refresh "
                            "and the iteration keeps the key holder's"}
        log("bootstrap of W and V at N=2^16 (%d levels per transform): %.3f s, output level %d, max|err| %.2e"
            % (BOOT_LEVELS, t_boot, ol, err))
        del kb, bt, ct, out_b, ws
        torch.cuda.empty_cache()
    out["bootstrap"] = boot_leg


    # the same iteration with W and V at the top of the chain (as a refresh that returned them there
    # would leave them; no bootstrap can): seconds per iteration from W = V = 0
    top_it = None
    if args.top_steps > 0 and work != top:
        run.reset(level=top)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.top_steps):
            run.step()
        torch.cuda.synchronize()
        top_it = {"level": top, "limbs": top + 1, "s_per_iter": round((time.perf_counter() - t0) / args.top_steps, 4),
                  "iterations": args.top_steps}
        if args.top_steps == 1:
            top_it["max_abs_dw_vs_fp64"] = float(abs(run.weights(cfg["n_features"] + 1) - w_fp64[1]).max())
        log("iteration with W and V at the top level %d: %.3f s" % (top, top_it["s_per_iter"]))
    out["top_level_iteration"] = top_it

    # the same iteration at the paper's working modulus: Table 1 gives Q = 2^275 for its ciphertexts
    # (4.6 MB encrypted blocks at N = 2^16), the modulus its weights and data carry through an
    # iteration; W and V at the lowest level of the chain whose modulus covers 2^275, trained for as
    # many iterations as the run above from W = V = 0: time per iteration and the decrypted model
    # against the main run's
    paper_q = None
    if args.paper_q_steps > 0:
        import numpy as np
        bits = np.cumsum(cfg["q_bits"])
        lq = int(np.argmax(bits >= 275))
        run.reset(level=lq)
        for _ in range(max(t_cmp - args.paper_q_steps, 0)):
            run.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.paper_q_steps):
            run.step()
        torch.cuda.synchronize()
        ps = (time.perf_counter() - t0) / args.paper_q_steps
        wq = run.weights(cfg["n_features"] + 1)
        paper_q = {"level": lq, "limbs": lq + 1, "log2_modulus": int(bits[lq]), "s_per_iter": round(ps, 4),
                   "iterations": int(run.state.t),
                   "max_abs_dw_vs_main_run": float(np.abs(wq - w_cmp).max()) if run.state.t == t_cmp else None,
                   "max_abs_dw_vs_fp64": float(np.abs(wq - w_fp64[t_cmp]).max()) if run.state.t == t_cmp else None,
                   "note": "Table 1's Q = 2^275: the working modulus of the paper's iteration"}
        log("iteration at level %d (2^%d): %.3f s, max|dw| vs the main run after %d iterations: %.2e" %
            (lq, bits[lq], ps, run.state.t, paper_q["max_abs_dw_vs_main_run"] or -1.0))
    out["paper_modulus_iteration"] = paper_q

    # the same task over the 1,024 x 32 partition of section 2.2 (7 column blocks; 10x fewer key
    # switches per iteration), trained for as many iterations as the run above from the same start:
    # its decrypted model against the 128 x 256 run's
    grid = None
    if args.grid_steps > 0:
        import numpy as np
        run = None
        torch.cuda.empty_cache()
        gcfg = synth.get_config("c3g")
        gr = EncryptedQGNAG(gcfg, data["X"], data["y"], batch=args.batch)
        for _ in range(max(t_cmp - args.grid_steps, 0)):
            gr.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.grid_steps):
            gr.step()
        torch.cuda.synchronize()
        gs = (time.perf_counter() - t0) / args.grid_steps
        wg = gr.weights(cfg["n_features"] + 1)
        grid = {"workload": gcfg["name"], "rows_per_block": gcfg["m"], "cols": gcfg["g"], "col_blocks": gr.nc,
                "ciphertexts": gr.Z.count, "s_per_iter": round(gs, 4), "iterations": int(gr.state.t),
                "max_abs_dw_vs_128x256": float(np.abs(wg - w_cmp).max()) if gr.state.t == t_cmp else None}
        log("grid 1024x32 iteration: %.3f s, max|dw| vs 128x256 after %d iterations: %.2e" %
            (gs, gr.state.t, grid["max_abs_dw_vs_128x256"]))
        if forms:
            # g8 and the learned forms, each trained from W = V = 0 for 10 iterations: validation
            # log-likelihood and AUROC of the decrypted model
            learned["layout_1024x32"] = {"iterations": 10}
            for name, co in forms.items():
                gr.set_sigmoid(co)
                gr.reset()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(10):
                    gr.step()
                torch.cuda.synchronize()
                dt = (time.perf_counter() - t0) / 10
                wl = gr.weights(cfg["n_features"] + 1)
                ll, auc = loglik_auroc(data["Xv"], data["yv"], wl)
                learned["layout_1024x32"][name] = {"s_per_iter": round(dt, 4), "valid_loglik": round(ll, 6),
                                                   "valid_auroc": round(auc, 6)}
                log("%s, 10 iterations on 1024 x 32: %.3f s/iter, valid loglik %.5f, AUROC %.5f" % (name, dt, ll, auc))
        del gr
        torch.cuda.empty_cache()
    out["grid_1024x32"] = grid


    # the paper's second workload (section 5.2, Table 2): MNIST-shaped, g16, 12 x 7 blocks; the quadratic
    # gradient beside the first-order NAG baseline (section 3.2, Fig. 1), decrypted log-likelihood and
    # validation AUROC after the same number of iterations
    mnist = None
    if args.mnist_steps > 0:
        mnist = mnist_leg(args.mnist_steps, args.batch)
    out["mnist_shaped"] = mnist

    # the paper's flow without the key holder (section 4.3 step 7; Table 1: one bootstrapping per
    # iteration) at paper scale: the same data and circuit on a chain of 50-bit primes (q0 = 2^60,
    # scale 2^50, sparse secret of weight 64), W and V at the level bootstrapping returns; each iteration
    # is followed by bootstrapping W and V together; decrypted weights against the FP64 run
    # (after every other leg: the main run's memory is released first)
    ni_leg = None
    if args.noninteractive_steps > 0:
        import numpy as np
        run = None
        torch.cuda.empty_cache()
        ncfg = dict(cfg, q_bits=NI_Q_BITS, p_bits=NI_P_BITS, log2_scale=NI_LOG2_SCALE)
        probe = heqg.Context.from_config(ncfg)
        _, _, ni_level, _ = probe.boot_shape(NI_R, NI_LEVELS)
        ni_steps = probe.boot_steps(NI_LEVELS)
        del probe
        nrun = EncryptedQGNAG(ncfg, data["X"], data["y"], batch=batch_used, level=ni_level,
                              secret_weight=BOOT_WEIGHT, extra_steps=ni_steps)
        nctx = nrun.ctx
        pts = nctx.boot_encode(NI_R, NI_LEVELS)
        nbt = nctx.boot_setup(pts, NI_R, BOOT_TAYLOR, levels=NI_LEVELS)
        del pts
        nws = heqg._ws(heqg.lib().heqg_boot_ws_bytes(nctx.h, NI_LEVELS, 2 * nrun.nc))
        upd_s, boot_s = [], []
        for _ in range(args.noninteractive_steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            nrun.step(refresh=False)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            nrun.bootstrap(nbt, nws)
            torch.cuda.synchronize()
            upd_s.append(t1 - t0)
            boot_s.append(time.perf_counter() - t1)
        k = args.noninteractive_steps
        w_ni = nrun.weights(cfg["n_features"] + 1)
        ref = heqg.plain_qgnag(data["X"], data["y"], k, coeffs=dict(nrun.coeffs), margins=False)[0]
        tail = slice(1, None) if k > 1 else slice(None)   # the first iteration also pays first-call setup
        ni_leg = {"iterations": k, "q_bits": "60 + 24 x 50", "special_primes": "7 x 60", "log2_scale": NI_LOG2_SCALE,
                  "work_level": ni_level, "double_angles": NI_R, "levels_per_transform": NI_LEVELS,
                  "taylor_degree": BOOT_TAYLOR, "secret_weight": BOOT_WEIGHT,
                  "update_s": round(float(np.mean(upd_s[tail])), 4), "bootstrap_s": round(float(np.mean(boot_s[tail])), 4),
                  "s_per_iter": round(float(np.mean(upd_s[tail]) + np.mean(boot_s[tail])), 4),
                  "max_abs_dw_vs_fp64": float(abs(w_ni - ref).max()),
                  "note": "50-bit primes take the 64-bit integer path (the FP64 path holds primes of at most 42 "
                          "bits), hence the slower update"}
        log("non-interactive: %d iterations with bootstrapping on the 50-bit chain (level %d): update %.3f s + "
            "bootstrap %.4f s per iteration, max|dw| vs FP64 %.2e" % (k, ni_level, ni_leg["update_s"],
                                                                    ni_leg["bootstrap_s"], ni_leg["max_abs_dw_vs_fp64"]))
        del nrun, nbt, nws, nctx
        torch.cuda.empty_cache()
    out["noninteractive"] = ni_leg

    if args.copy_probe:
        src = torch.ones(1 << 27, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(cfg, data, n_blocks, work)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
