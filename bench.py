"""Benchmark: the online guiding frame loop on one MI355X.

One step = one frame of a 1-spp path tracer's guiding work: NASG queries
(MLP forward + decode + sample + pdf) for 2^20, 600000, 300000 and 120000
vertices (four bounces), then one training step (fused forward recompute +
weighted-NLL backward + Adam) on 2^18 samples, with the BF16 network
9 -> 64 x 4 -> 8*16 (K = 16 NASG lobes). Inputs are synthetic, seeded and
resident in HBM before timing; the frames cycle through 8 sets of distinct
inputs (8 x 121 MB, more than the last-level cache holds), each set's frame
captured once as a HIP graph and replayed in turn. Prints one JSON line.

Also measured: the same frame with the FP32 network, the stand-alone
nasg_pdf / nasg_sample kernels on stored records (2^20 vertices), the query
kernel's roofline (HIP events around repeated launches), and the FP64
oracle on the host CPU for a bounded sample of the frame.
"""

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "NASG queries/s (fwd+sample+pdf) & train samples/s (fwd+bwd), bf16 vs fp32"
BOUNCES = (1 << 20, 600000, 300000, 120000)
TRAIN_B = 1 << 18
H, NH, K = 64, 4, 16

# MI355X published peaks used for the roofline fractions
PEAK_HBM_GBS = 8000.0
PEAK_BF16_TFLOPS = 2500.0
# VALU issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one FP32 op per
# lane per cycle; transcendentals take four such slots)
PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12


def query_valu_ops(k):
    """Algorithmic VALU op-slots of one query with k lobes (cost model:
    add/mul/fma/compare/select = 1 slot, exp2/log2/rcp/rsqrt/sqrt/sin/cos = 4).
    Per lobe 180: decode of five sin/cos values 50, sin theta 6, the two pair
    normalisations 16, frame 7, lambda and a 14, log K 20, mixture weight 9,
    lobe value at the sampled direction with its log-sum-exp term 55, CDF 3.
    Per vertex 100: direct sampling 88, normalising the direction 8,
    cross-lane reductions and stores 4."""
    return 180 * k + 100


def mlp_flops(hidden, n_hidden, k):
    macs = hidden * 10 + (n_hidden - 1) * hidden * hidden + 8 * k * hidden
    return 2 * macs


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-fp32", action="store_true")
    p.add_argument("--no-graph", action="store_true")
    p.add_argument("--no-configs", action="store_true")
    p.add_argument("--only", choices=["frame", "query", "records", "train", "copy", "c5", "paper", "paper_query",
                                      "paper_train"], default=None,
                   help="run one leg only (for profilers)")
    return p.parse_args()


# Frames of distinct inputs that the frame loop cycles through: 8 x 121 MB
# of vertices and training samples, so that no frame finds its inputs in the
# 256 MB last-level cache (a renderer streams new vertices every frame)
SLICES = 8


class Frame:
    """Device-resident inputs of SLICES frames and the launch sequence of one
    frame; frame i reads slice i mod SLICES."""

    def __init__(self, precision, seed=1000, n_slices=SLICES):
        import torch
        from paper_2303_08064_amd import synth
        from paper_2303_08064_amd.nasg import NasgGuide
        self.torch = torch
        mats = synth.init_weights(synth.layer_shapes(H, NH, K), synth.rng_for(42))
        self.guide = NasgGuide(synth.flat_weights(mats), hidden=H, n_hidden=NH, n_lobes=K,
                               precision=precision, lr=1e-3, max_batch=TRAIN_B)
        rng = synth.rng_for(seed)
        dev = "cuda"
        tgt = synth.VmfTarget(4, seed=1001)
        self.slices = []
        for _ in range(n_slices):
            q_in = [(torch.from_numpy(synth.features(n, rng)).to(dev),
                     torch.from_numpy(synth.uniforms(n, rng)).to(dev)) for n in BOUNCES]
            f, d, w = synth.training_batch(TRAIN_B, rng, tgt)
            t_in = (torch.from_numpy(f).to(dev), torch.from_numpy(d).to(dev), torch.from_numpy(w).to(dev))
            self.slices.append((q_in, t_in))
        self.q_in, self.t_in = self.slices[0]
        self.q_out = [(torch.empty(3, n, device=dev), torch.empty(n, device=dev)) for n in BOUNCES]
        torch.cuda.synchronize()

    def run(self, i=0):
        g = self.guide
        q_in, t_in = self.slices[i % len(self.slices)]
        for (f, xi), (d, p) in zip(q_in, self.q_out):
            g.query(f, xi, dir_out=d, pdf_out=p)
        g.train_step(*t_in)


# The paper's default configuration (Sec. 4.1, Sec. 6): 4 hidden layers of
# 128 units on the encoded input, K = 8 lobes plus the selection output, and
# S = 2^16 training samples per frame taken as T = 16 steps of t = 4096 (Sec. 5)
PAPER_T, PAPER_TB = 16, 4096


class PaperFrame:
    """One frame of the paper's default configuration: the same four bounces
    of queries, then T Adam steps of t samples each on the blended loss;
    frame i reads the i mod n_slices-th set of inputs, as in Frame."""

    def __init__(self, seed=3000, precision="bf16", n_slices=SLICES):
        import torch
        from paper_2303_08064_amd import synth
        from paper_2303_08064_amd.nasg import NasgGuide
        self.torch = torch
        mats = synth.init_weights(synth.layer_shapes(128, 4, 8, selection=True, encoded=True), synth.rng_for(42))
        self.guide = NasgGuide(synth.flat_weights(mats), hidden=128, n_hidden=4, n_lobes=8, precision=precision,
                               lr=1e-3, max_batch=PAPER_TB, selection=True, mis_fraction=0.2, encoded=True)
        rng = synth.rng_for(seed)
        dev = "cuda"
        tgt = synth.VmfTarget(4, seed=1001)
        self.slices = []
        for _ in range(n_slices):
            q_in = [(torch.from_numpy(synth.features(n, rng)).to(dev),
                     torch.from_numpy(synth.uniforms(n, rng)).to(dev)) for n in BOUNCES]
            t_in = []
            for _ in range(PAPER_T):
                f, d, w = synth.training_batch(PAPER_TB, rng, tgt)
                pdf = synth.lambert_pdf(d, f[6:9])
                t_in.append(tuple(torch.from_numpy(x).to(dev) for x in (f, d, w, pdf)))
            self.slices.append((q_in, t_in))
        self.q_in, self.t_in = self.slices[0]
        self.q_out = [(torch.empty(3, n, device=dev), torch.empty(n, device=dev), torch.empty(n, device=dev))
                      for n in BOUNCES]
        torch.cuda.synchronize()

    def run(self, i=0):
        g = self.guide
        q_in, t_in = self.slices[i % len(self.slices)]
        for (f, xi), (d, p, c) in zip(q_in, self.q_out):
            g.query(f, xi, dir_out=d, pdf_out=p, sel_out=c)
        for f, d, w, pdf in t_in:
            g.train_step(f, d, w, bsdf_pdf=pdf)


def paper_leg(steps, use_graph, fp32=True):
    """The paper's default configuration, timed like the main frame, plus
    its query and single training step on their own, and the same frame
    with the FP32 network."""
    import torch
    fr = PaperFrame()
    ms, _ = time_frames(fr, steps, 2, use_graph)
    g = fr.guide
    (f, xi), (d, p, c) = fr.q_in[0], fr.q_out[0]
    ms_q = kernel_avg_ms(lambda: g.query(f, xi, dir_out=d, pdf_out=p, sel_out=c), 10)
    # the MLP alone: the raw forward of the same 2^20 vertices (no NASG work)
    raw = torch.empty(g.n_out, f.shape[1], dtype=torch.float32, device=f.device)
    ms_f = kernel_avg_ms(lambda: g.forward_raw(f, out=raw), 10)
    del raw
    f0, d0, w0, p0 = fr.t_in[0]
    ms_t = kernel_avg_ms(lambda: g.train_step(f0, d0, w0, bsdf_pdf=p0), 20)
    nq = sum(BOUNCES)
    ns = PAPER_T * PAPER_TB
    q_fl = mlp_flops_net(128, 4, 8, 64, 1)
    extra = {}
    if fp32:
        del fr
        f32 = PaperFrame(precision="f32")
        ms32, _ = time_frames(f32, max(3, steps // 4), 1, use_graph)
        extra = {"fp32_ms_per_frame": round(ms32, 4), "speedup_bf16": round(ms32 / ms, 3)}
        del f32
    return {
        "workload": "paper default: encoded input (one-blob 57 + omega_o + n + 1 = 64) -> 128x4 -> 8*8+1 "
                    "(K=8 with selection), BF16; queries 2^20+600000+300000+120000 and 16 Adam steps of "
                    f"4096 samples (S = 2^16, blended loss) per frame, HIP graph replay; frames cycle through "
                    f"{SLICES} sets of distinct inputs",
        "ms_per_frame": round(ms, 4), "queries_per_s": round(nq / (ms * 1e-3), 1),
        "train_samples_per_s": round(ns / (ms * 1e-3), 1),
        "query_2e20_ms": round(ms_q, 4), "query_mfma_tflops": round(q_fl * (1 << 20) / (ms_q * 1e-3) / 1e12, 1),
        "forward_2e20_ms": round(ms_f, 4),
        "forward_mfma_frac_bf16": round(q_fl * (1 << 20) / (ms_f * 1e-3) / 1e12 / PEAK_BF16_TFLOPS, 4),
        "train_step_4096_us": round(ms_t * 1e3, 1),
        **extra,
    }


def mlp_flops_net(hidden, n_hidden, k, n_in, sel):
    """Forward MFMA FLOPs of one vertex: n_in inputs (with the one), n_hidden
    layers of `hidden`, 8k + sel outputs."""
    return 2 * (hidden * n_in + (n_hidden - 1) * hidden * hidden + (8 * k + sel) * hidden)


def time_frames(frame, steps, warmup, use_graph):
    """Milliseconds per frame over `steps` frames after `warmup` untimed ones.
    With use_graph, each slice's frame is captured once as a HIP graph and the
    graphs are replayed in turn (frame i: slice i mod the number of slices)."""
    import torch
    n_slices = len(getattr(frame, "slices", [None]))
    for i in range(warmup):
        frame.run(i) if n_slices > 1 else frame.run()
    torch.cuda.synchronize()
    replays = [(lambda i=i: frame.run(i)) for i in range(n_slices)] if n_slices > 1 else [frame.run]
    if use_graph:
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        graphs = []
        with torch.cuda.stream(s):
            for run in replays:
                run()   # one more eager pass on the capture stream
                torch.cuda.synchronize()
                graph = torch.cuda.CUDAGraph()
                with torch.cuda.graph(graph, stream=s):
                    run()
                graphs.append(graph)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        replays = [g.replay for g in graphs]
        for r in replays:
            r()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(steps):
        replays[i % len(replays)]()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / steps
    return ms, wall


def kernel_avg_ms(fn, reps):
    """Average duration of fn's launches, by HIP events on the launching stream."""
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def source_hash(names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2303_08064_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


QUERY_SOURCES = ["query.hip", "mlp.hpp", "nasg_math.hpp", "common.hpp", "kernels.hpp", "layout.hpp", "epilogue.hpp"]


def committed_traffic():
    """HBM bytes per query launch from the committed counter summary, if it was
    taken on the current query-kernel sources (its `source_hash:` line)."""
    p = os.path.join(ROOT, "profiles", "query_bf16_k16_1m_counters.txt")
    if not os.path.exists(p):
        return None
    fields = {}
    with open(p) as f:
        for line in f:
            key, sep, val = line.partition(":")
            if sep and key.strip() in ("source_hash", "hbm_bytes_per_launch"):
                fields[key.strip()] = val.strip()
    if fields.get("source_hash") != source_hash(QUERY_SOURCES) or "hbm_bytes_per_launch" not in fields:
        return None
    return int(fields["hbm_bytes_per_launch"])


def query_launch_ms(frame, warm=100, reps=20):
    """Average duration of the 2^20-vertex query launch: `warm` launches
    first (the GPU's clocks settle under load), then `reps` timed by HIP
    events on the launching stream. `--only query` runs exactly this, so the
    rocprofv3 kernel trace of that command averages the same launches."""
    import torch
    g = frame.guide
    (f, xi), (d, p) = frame.q_in[0], frame.q_out[0]
    run = lambda: g.query(f, xi, dir_out=d, pdf_out=p)
    for _ in range(warm):
        run()
    torch.cuda.synchronize()
    return kernel_avg_ms(run, reps)


def query_roofline(frame, reps=20):
    import torch
    (f, xi) = frame.q_in[0]
    ms = query_launch_ms(frame, reps=reps)
    n = f.shape[1]
    ops = query_valu_ops(K) * n
    achieved = ops / (ms * 1e-3) / 1e12
    mfma = mlp_flops(H, NH, K) * n / (ms * 1e-3) / 1e12
    hbm = (9 + 4 + 3 + 1) * 4 * n / (ms * 1e-3) / 1e9
    torch.cuda.synchronize()
    return {
        "kernel": "query_kernel<64,16,bf16> (nasg_query, 2^20 vertices)",
        "bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_VALU_TOPS, 3),
        "unit": "TOP/s (VALU op-slots)", "frac": round(achieved / PEAK_VALU_TOPS, 4),
        "traffic": committed_traffic(), "avg_ms": round(ms, 4),
        "mfma_tflops": round(mfma, 2), "mfma_frac_bf16": round(mfma / PEAK_BF16_TFLOPS, 4),
        "hbm_gbs_algorithmic": round(hbm, 1),
    }


def records_legs(frame, reps=20):
    import torch
    from paper_2303_08064_amd import synth
    from paper_2303_08064_amd.nasg import record_elems
    g = frame.guide
    (f, xi), (d, p) = frame.q_in[0], frame.q_out[0]
    n = f.shape[1]
    rec = torch.empty(record_elems(K, n), device="cuda")
    g.query(f, xi, dir_out=d, pdf_out=p, rec_out=rec)
    xi2 = torch.from_numpy(synth.uniforms(n, synth.rng_for(77))).cuda()
    pdf_out = torch.empty(n, device="cuda")
    d2, p2 = torch.empty(3, n, device="cuda"), torch.empty(n, device="cuda")
    ms_pdf = kernel_avg_ms(lambda: g.pdf(rec, d, pdf_out=pdf_out), reps)
    ms_smp = kernel_avg_ms(lambda: g.sample(rec, xi2, dir_out=d2, pdf_out=p2), reps)
    rec_bytes = 9 * K * 4
    b_pdf = (rec_bytes + 12 + 4) * n
    b_smp = (rec_bytes + 16 + 12 + 4) * n
    return {
        "pdf": {"avg_ms": round(ms_pdf, 4), "gbs": round(b_pdf / (ms_pdf * 1e-3) / 1e9, 1),
                "frac_hbm": round(b_pdf / (ms_pdf * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)},
        "sample": {"avg_ms": round(ms_smp, 4), "gbs": round(b_smp / (ms_smp * 1e-3) / 1e9, 1),
                   "frac_hbm": round(b_smp / (ms_smp * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)},
        "vertices": n,
    }


def train_leg(frame, reps=10):
    g = frame.guide
    ms = kernel_avg_ms(lambda: g.train_step(*frame.t_in), reps)
    return {"avg_ms": round(ms, 4), "samples_per_s": round(TRAIN_B / (ms * 1e-3), 1)}


def stage_legs(frame, reps=10):
    """Microseconds per stage of one frame, each stage launched on its own:
    the query of every bounce, then the training step."""
    g = frame.guide
    out = {}
    for (f, xi), (d, p), n in zip(frame.q_in, frame.q_out, BOUNCES):
        out[f"query_{n}"] = round(kernel_avg_ms(lambda: g.query(f, xi, dir_out=d, pdf_out=p), reps) * 1e3, 1)
    out[f"train_step_{TRAIN_B}"] = round(kernel_avg_ms(lambda: g.train_step(*frame.t_in), reps) * 1e3, 1)
    return out


PEAK_F32_MFMA_TFLOPS = 157.3


def train_flops(hidden, n_hidden, k):
    """Algorithmic MFMA FLOPs of one training sample: forward, dgrad through
    layers L..1 (none into the input) and the weight gradient of every layer."""
    fwd = mlp_flops(hidden, n_hidden, k)
    dgrad = 2 * ((n_hidden - 1) * hidden * hidden + 8 * k * hidden)
    return fwd + dgrad + fwd


def config_legs():
    """The other workload configurations, each timed briefly on its own:
    C1 one small FP32 step (latency), C2 FP32 training on 2^18 samples, C3
    BF16 and FP32 inference on 2^20 queries, C5 BF16 training of the large
    network on 2^22 samples."""
    import torch
    from paper_2303_08064_amd import synth
    from paper_2303_08064_amd.nasg import NasgGuide
    out = {}

    def guide(hidden, n_hidden, k, prec, max_batch):
        mats = synth.init_weights(synth.layer_shapes(hidden, n_hidden, k), synth.rng_for(42))
        return NasgGuide(synth.flat_weights(mats), hidden=hidden, n_hidden=n_hidden, n_lobes=k,
                         precision=prec, max_batch=max_batch)

    def batch(n, seed, target):
        f, d, w = synth.training_batch(n, synth.rng_for(seed), target)
        return torch.from_numpy(f).cuda(), torch.from_numpy(d).cuda(), torch.from_numpy(w).cuda()

    vmf = synth.VmfTarget(4, seed=1001)
    # C1: 9->64->64->64->8*4, FP32, 4096 vertices, one fwd+NLL+bwd+Adam step
    g = guide(64, 3, 4, "f32", 4096)
    b = batch(4096, 1000, vmf)
    ms = kernel_avg_ms(lambda: g.train_step(*b), 50)
    out["c1_fp32_step"] = {"us_per_step": round(ms * 1e3, 1), "batch": 4096}
    del g, b
    # C2: 9->64x4->8*8, FP32, 2^18 samples per step
    n = 1 << 18
    g = guide(64, 4, 8, "f32", n)
    b = batch(n, 1001, vmf)
    ms = kernel_avg_ms(lambda: g.train_step(*b), 10)
    fl = train_flops(64, 4, 8) * n / (ms * 1e-3) / 1e12
    out["c2_fp32_train"] = {"samples_per_s": round(n / (ms * 1e-3), 1), "ms_per_step": round(ms, 4),
                            "mfma_tflops": round(fl, 2), "frac_fp32_mfma": round(fl / PEAK_F32_MFMA_TFLOPS, 4)}
    del g, b
    # C3: 9->64x4->8*16, 2^20 queries, BF16 and FP32 MLP
    n = 1 << 20
    rng = synth.rng_for(1002)
    f = torch.from_numpy(synth.features(n, rng)).cuda()
    xi = torch.from_numpy(synth.uniforms(n, rng)).cuda()
    d, p = torch.empty(3, n, device="cuda"), torch.empty(n, device="cuda")
    for prec in ("bf16", "f32"):
        g = guide(64, 4, 16, prec, 1)
        ms = kernel_avg_ms(lambda: g.query(f, xi, dir_out=d, pdf_out=p), 20)
        out[f"c3_{prec}_query"] = {"queries_per_s": round(n / (ms * 1e-3), 1), "ms": round(ms, 4)}
        del g
    del f, xi, d, p
    # C5: 9->128x4->8*32, 2^22 samples per step, anisotropic target; BF16
    # (the configuration's precision) and FP32 (its comparison)
    n = 1 << 22
    b = batch(n, 1004, synth.AnisoTarget(8, seed=1005))
    for prec, peak in (("bf16", PEAK_BF16_TFLOPS), ("f32", PEAK_F32_MFMA_TFLOPS)):
        g = guide(128, 4, 32, prec, n)
        ms = kernel_avg_ms(lambda: g.train_step(*b), 3 if prec == "bf16" else 1)
        fl = train_flops(128, 4, 32) * n / (ms * 1e-3) / 1e12
        out[f"c5_{prec}_train"] = {"samples_per_s": round(n / (ms * 1e-3), 1), "ms_per_step": round(ms, 3),
                                   "mfma_tflops_algorithmic": round(fl, 1),
                                   f"frac_{prec}_mfma": round(fl / peak, 4)}
        del g
    del b
    torch.cuda.synchronize()
    return out


def cpu_baseline(min_seconds=10.0, max_pieces=64, fraction=8):
    """The FP64 oracle on the host for a bounded sample of the frame: pieces
    of 1/fraction of a frame (every bounce's queries and the training samples
    scaled by 1/fraction, plus one Adam step each) until min_seconds have
    passed; reported in queries/s of whole frames."""
    import torch
    from oracle import mlp as omlp, nasg as onasg, train as otrain
    from paper_2303_08064_amd import synth
    mats = synth.init_weights(synth.layer_shapes(H, NH, K), synth.rng_for(42))
    W = [torch.tensor(m, dtype=torch.float64) for m in mats]
    flatW = torch.cat([x.reshape(-1) for x in W])
    rng = synth.rng_for(2000)
    tgt = synth.VmfTarget(4, seed=1001)
    nq = [n // fraction for n in BOUNCES]
    nt = TRAIN_B // fraction
    chunk = 65536
    pieces = 0
    dt = 0.0   # oracle compute time only; host generation of inputs is not timed
    while pieces < max_pieces and (pieces == 0 or dt < min_seconds):
        for n in nq:
            for s in range(0, n, chunk):
                m = min(chunk, n - s)
                f, xi = synth.features(m, rng), synth.uniforms(m, rng)
                t0 = time.perf_counter()
                lob = onasg.decode(omlp.forward(W, f.T, bf16=True), K)
                v, _ = onasg.sample(lob, xi.T.astype(np.float64))
                onasg.mixture_log_pdf(v, lob)
                dt += time.perf_counter() - t0
        grads = None
        for s in range(0, nt, chunk):
            m = min(chunk, nt - s)
            f, d, w = synth.training_batch(m, rng, tgt)
            t0 = time.perf_counter()
            _, gl = otrain.loss_and_grad(W, f.T, d.T, w.astype(np.float64), K, bf16=True)
            grads = gl if grads is None else [a + b for a, b in zip(grads, gl)]
            dt += time.perf_counter() - t0
        t0 = time.perf_counter()
        flat = torch.cat([x.reshape(-1) for x in grads])
        z = torch.zeros_like(flat)
        otrain.adam_step(flatW, flat, z, z.clone(), 0, 1e-3)
        dt += time.perf_counter() - t0
        pieces += 1
    frames_per_s = (pieces / fraction) / dt
    # the same oracle on one thread, for one piece of 1/64 of a frame
    threads = torch.get_num_threads()
    torch.set_num_threads(1)
    t1 = 0.0
    for n in [n // 64 for n in BOUNCES]:
        f, xi = synth.features(n, rng), synth.uniforms(n, rng)
        t0 = time.perf_counter()
        lob = onasg.decode(omlp.forward(W, f.T, bf16=True), K)
        v, _ = onasg.sample(lob, xi.T.astype(np.float64))
        onasg.mixture_log_pdf(v, lob)
        t1 += time.perf_counter() - t0
    torch.set_num_threads(threads)
    return {"value": round(frames_per_s * sum(BOUNCES), 1), "unit": "queries/s", "cores": threads,
            "one_thread_query_path_per_s": round(sum(n // 64 for n in BOUNCES) / t1, 1),
            "kind": "oracle", "seconds": round(dt, 2),
            "train_samples_per_s": round(frames_per_s * TRAIN_B, 1),
            "sample": f"{pieces} x 1/{fraction} of a frame (each: {sum(nq)} queries, bounces {nq}, "
                      f"{nt} training samples, one Adam step); FP64 with BF16-rounded MLP operands; "
                      f"only the oracle's compute is timed; one_thread_query_path_per_s: the query path "
                      f"alone (no training) on one thread over 1/64 of a frame's queries"}


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the guiding hot path is data-parallel over vertices, "
              "and the figure reported is one GPU's throughput on its share of a frame.", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    # the single-kernel legs read one set of inputs; the frame loop cycles through SLICES
    frame = Frame("bf16", n_slices=SLICES if a.only in (None, "frame") else 1)
    if a.only == "query":
        ms = query_launch_ms(frame, reps=a.steps)
        print(json.dumps({"only": "query", "steps": a.steps, "avg_ms": round(ms, 4)}))
        return
    if a.only == "copy":
        # a plain device copy of known size, to scale the HBM byte counters
        n = 64 << 20
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(a.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"only": "copy", "bytes_read": 4 * n, "bytes_written": 4 * n, "steps": a.steps}))
        return
    if a.only == "c5":
        from paper_2303_08064_amd import synth
        from paper_2303_08064_amd.nasg import NasgGuide
        n = 1 << 22
        mats = synth.init_weights(synth.layer_shapes(128, 4, 32), synth.rng_for(42))
        g = NasgGuide(synth.flat_weights(mats), hidden=128, n_hidden=4, n_lobes=32, precision="bf16", max_batch=n)
        f, d, w = synth.training_batch(n, synth.rng_for(1004), synth.AnisoTarget(8, seed=1005))
        b = (torch.from_numpy(f).cuda(), torch.from_numpy(d).cuda(), torch.from_numpy(w).cuda())
        g.train_step(*b)
        ms = kernel_avg_ms(lambda: g.train_step(*b), a.steps)
        print(json.dumps({"only": "c5", "steps": a.steps, "ms_per_step": round(ms, 4)}))
        return
    if a.only in ("paper_query", "paper_train"):
        fr = PaperFrame(n_slices=1)
        (f, xi), (d, p, c) = fr.q_in[0], fr.q_out[0]
        for _ in range(a.steps):
            if a.only == "paper_query":
                fr.guide.query(f, xi, dir_out=d, pdf_out=p, sel_out=c)
            else:
                fr.guide.train_step(*fr.t_in[0][:3], bsdf_pdf=fr.t_in[0][3])
        torch.cuda.synchronize()
        print(json.dumps({"only": a.only, "steps": a.steps}))
        return
    if a.only == "paper":
        print(json.dumps({"only": "paper", **paper_leg(a.steps, not a.no_graph, fp32=not a.no_fp32)}))
        return
    if a.only == "records":
        print(json.dumps({"only": "records", **records_legs(frame, a.steps)}))
        return
    if a.only == "train":
        print(json.dumps({"only": "train", **train_leg(frame, a.steps)}))
        return
    ms, wall = time_frames(frame, a.steps, a.warmup, not a.no_graph)
    nq = sum(BOUNCES)
    out = {
        "metric": METRIC,
        "value": round(nq / (ms * 1e-3), 1),
        "unit": "queries/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "online guiding frame loop: NASG MLP 9->64x4->8*16 (K=16), queries "
                               "2^20+600000+300000+120000 (fwd+sample+pdf) and one 2^18-sample training "
                               "step (fwd+bwd+Adam) per frame, HIP graph replay; frames cycle through "
                               f"{SLICES} sets of distinct inputs ({SLICES} x 121 MB, past the last-level cache)",
                   "queries_per_frame": nq, "train_samples_per_frame": TRAIN_B,
                   "hidden": H, "n_hidden": NH, "n_lobes": K, "precision": "bf16"},
        "train_samples_per_s": round(TRAIN_B / (ms * 1e-3), 1),
        "frames_per_s": round(1e3 / ms, 2),
        "wall_s_timed": round(wall, 3),
    }
    if a.only != "frame":
        out["roofline"] = query_roofline(frame)
        out["records"] = records_legs(frame)
        out["train_step"] = train_leg(frame)
        out["frame_stages_us"] = stage_legs(frame)
    if not a.no_configs and a.only != "frame":
        out["configs"] = config_legs()
        out["configs"]["paper_default_frame"] = paper_leg(10, not a.no_graph)
    if not a.no_fp32 and a.only != "frame":
        f32 = Frame("f32")
        ms32, _ = time_frames(f32, max(5, a.steps // 5), 2, not a.no_graph)
        out["fp32"] = {"ms_per_step": round(ms32, 4), "value": round(nq / (ms32 * 1e-3), 1),
                       "train_samples_per_s": round(TRAIN_B / (ms32 * 1e-3), 1),
                       "speedup_bf16": round(ms32 / ms, 3)}
        del f32
    if not a.no_cpu_baseline and a.only != "frame":
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
