"""Decode-path benchmark: decoded Mpixel/s of the GPU decode path (context
model + CDF tables + inverse lifting), p50/p99 latency, on one GPU.

One step = one coder-elided decode of the 512x768 three-plane YCbCr image:
for each of the 13 subbands x 4 coding steps, the context model, the CDF
tables of that step and the scatter of that step's symbols (the symbols the
host entropy coder would return are taken from a device buffer), then
dequantisation and synthesis.  Inputs are resident in HBM before timing.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MFMA_PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0}   # MI355X dense matrix peaks
HBM_PEAK_GBS = 8000.0


def context_flops_per_coef(cfg):
    """Algorithmic FLOPs of the context model per coefficient (all 4 steps).

    ConvLSTM: 9 (1 + C) 4C MACs at every position.  Step stacks: every layer
    but the last at all positions, the 3K-output head at the quarter of
    positions its step codes: sum_g [9 Cin_g C + (L - 2) 9 C^2 + 9 C 3K / 4].
    """
    C, Lc, K = cfg["ctx_ch"], cfg["ctx_layers"], cfg["mix_k"]
    lstm = 9 * (1 + C) * 4 * C
    stacks = 0
    for g in range(4):
        cin = C if g == 0 else C + 1
        stacks += 9 * cin * C + (Lc - 2) * 9 * C * C + 9 * C * 3 * K / 4.0
    return 2.0 * (lstm + stacks)


def cpu_baseline(cfg, w, x, q_planes):
    """The FP64 oracle's decode path on plane 0 only (a third of one image)."""
    import oracle as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count()
    H, W = x.shape[1:]
    qs = O.unpack(q_planes[:1], cfg, H, W)
    t0 = time.perf_counter()
    O.decode_path(qs, cfg, w)
    dt = time.perf_counter() - t0
    mpx = (H * W / 3.0) / dt / 1e6     # one of three planes = a third of the image's pixels
    return dict(value=round(mpx, 6), unit="Mpixel/s", cores=int(threads), kind="oracle",
                seconds=round(dt, 3),
                sample=f"plane 0 of the {H}x{W}x3 image: context model of all 52 steps, CDF tables "
                       "and synthesis in float64 (one third of one image's work)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=["fp32", "bf16"], default="fp32",
                    help="context-conv precision (lifting and CDFs stay FP32)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU; this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2405_12631_amd import codec
    from wvgen import get_config, make_weights, pack_weights, sinusoid_1f_planes

    cfg = get_config("ycbcr512x768")
    H, W, N = cfg["H"], cfg["W"], cfg["planes"]
    w = make_weights(cfg)
    from paper_2405_12631_amd import WV_BF16, WV_FP32
    prec = WV_BF16 if args.precision == "bf16" else WV_FP32
    model = codec.Model(cfg, pack_weights(cfg, w), precision=prec)
    x = sinusoid_1f_planes(H, W, planes=N, seed=cfg["seed_image"])
    ws = codec.Workspace(model, N, H, W)
    q_known, _, _ = codec.analyze(model, torch.from_numpy(x).cuda(), ws)
    syms = codec.prepare_elided(model, q_known, ws)
    q = torch.zeros_like(q_known)
    xhat = torch.empty((N, H, W), dtype=torch.float32, device="cuda")
    nsub = len(ws.lay)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        q.zero_()
        for i in range(nsub):
            for g in range(4):
                if ev is not None:
                    ev[0].append(torch.cuda.Event(enable_timing=True))
                    ev[0][-1].record(stream)
                prm = codec.context_params(model, q, ws, i, g)
                if ev is not None:
                    ev[1].append(torch.cuda.Event(enable_timing=True))
                    ev[1][-1].record(stream)
                codec.cdf_tables(model, prm, out=ws.cdf)
                codec.scatter_symbols(model, syms[i][g], q, ws, i, g)
        if ev is not None:
            ev[2].append(torch.cuda.Event(enable_timing=True))
            ev[2][-1].record(stream)
        codec.synthesize(model, ws, q=q, xhat=xhat)
        if ev is not None:
            ev[3].append(torch.cuda.Event(enable_timing=True))
            ev[3][-1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    assert torch.equal(q, q_known), "decode did not reproduce the symbols"

    ev = ([], [], [], [])
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        step(ev)
        ends[k].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    lat = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])
    ctx_ms = np.array([a.elapsed_time(b) for a, b in zip(ev[0], ev[1])]).reshape(args.steps, -1)
    syn_ms = np.array([a.elapsed_time(b) for a, b in zip(ev[2], ev[3])])
    ms_step = elapsed * 1e3 / args.steps
    mpx = H * W * args.steps / elapsed / 1e6

    ctx_flops = context_flops_per_coef(cfg) * H * W * N
    ctx_time = ctx_ms.sum(axis=1).mean() * 1e-3
    n_ctx_launch = nsub * (cfg["ctx_layers"] * 4) + nsub      # step layers + one LSTM per subband
    peak = MFMA_PEAK_TFLOPS[args.precision]
    kname = "conv3x3_mfma_bf16" if args.precision == "bf16" else "conv3x3_mfma_f32"
    roof = dict(bound="mfma", achieved=round(ctx_flops / ctx_time / 1e12, 3),
                peak=peak, unit="TFLOP/s",
                frac=round(ctx_flops / ctx_time / 1e12 / peak, 4), traffic=None,
                kernel=f"{kname} (context model: ConvLSTM + step stacks)",
                flops_per_decode=ctx_flops, launches_per_decode=n_ctx_launch,
                avg_launch_us=round(ctx_time / n_ctx_launch * 1e6, 2))

    out = dict(
        metric="decoded Mpixel/s (ctx model+CDF+inverse lifting), p50/p99 latency vs plain FP32",
        value=round(mpx, 4), unit="Mpixel/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=round(ms_step, 3), higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f32" if args.precision == "fp32" else "bf16 context convs (fp32 accumulate), fp32 lifting/cdf",
        data="synthetic",
        config=dict(workload="ycbcr512x768: one 512x768 3-plane YCbCr image, 1/f sinusoids + noise "
                             "(seed 2), 4-level CNN lifting (32 ch), 64-ch 4-layer context stacks, "
                             f"K=3 mixture, step 4, {args.precision.upper()} context, batch 1, "
                             "coder elided",
                    batch=1, planes=N, H=H, W=W),
        p50_ms=round(float(np.percentile(lat, 50)), 3), p99_ms=round(float(np.percentile(lat, 99)), 3),
        stage_ms=dict(context=round(float(ctx_ms.sum(1).mean()), 3),
                      synthesis=round(float(syn_ms.mean()), 3),
                      cdf_scatter_rest=round(float(lat.mean() - ctx_ms.sum(1).mean() - syn_ms.mean()), 3)),
        roofline=roof,
    )
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, w, x, q_known.cpu().numpy().astype(np.int64))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
