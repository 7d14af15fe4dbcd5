"""Small workload driver for rocprofv3 runs.

    python -m paper_1610_04124_amd.profile_driver --mode batch --launches 3
    python -m paper_1610_04124_amd.profile_driver --mode frame --launches 3
    python -m paper_1610_04124_amd.profile_driver --mode copy

batch: the persistent batched launch over 64 synthetic 1024x440 frames
       (stixel width 5), replayed from a HIP graph;
hires: the same over 16 frames of 2048x880 (stixel width 5, d_range 256);
frame: the per-frame path (three kernels) on the same frames;
copy:  a plain 256 MiB device-to-device copy, whose FETCH_SIZE / WRITE_SIZE
       readings calibrate the HBM byte counters.
"""

from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mode", choices=["batch", "hires", "frame", "copy"], default="batch")
    ap.add_argument("--launches", type=int, default=3)
    ap.add_argument("--frames", type=int, default=64)
    ap.add_argument("--waves", type=int, default=0,
                    help="waves per column (0: automatic per frame, one per column batched)")
    ap.add_argument("--workgroups", type=int, default=0,
                    help="resident workgroups of the batched launch (0: the occupancy limit)")
    ap.add_argument("--placement", type=int, default=0,
                    help="object prefix table placement (frame mode): 0 auto, 1 HBM, 2 LDS")
    args = ap.parse_args()

    import torch

    dev = torch.device("cuda", 0)
    if args.mode == "copy":
        n = 256 * 1024 * 1024 // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(args.launches):
            b.copy_(a)
        torch.cuda.synchronize()
        print(f"copied {n * 4} bytes x {args.launches}", flush=True)
        return

    import synth
    import paper_1610_04124_amd as P

    if args.mode == "hires":
        W, H, D, nframes = 2048, 880, 256, min(args.frames, 16)
        cam = synth.camera_for_size(W, H)
        params = synth.make_params(camera=cam, max_width=W, max_height=H, max_disparity=D)
        specs = [synth.SceneSpec(W, H, D, cam, seed=i) for i in range(nframes)]
    else:
        W, H, D, nframes = 1024, 440, 128, args.frames
        params = synth.make_params()
        specs = [synth.SceneSpec(seed=i) for i in range(nframes)]
    h = P.Stixels(params)
    h.set_waves(args.waves)
    h.set_po_placement(args.placement)
    frames = [torch.from_numpy(synth.generate_frame(sp)).to(dev) for sp in specs]
    outs = [h.new_output(W, H) for _ in frames]
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    if args.mode in ("batch", "hires"):
        b = P.Batch(len(frames), len(frames) * (W // 5), H, D, args.workgroups)
        b.set_waves(args.waves)
        b.capture(list(zip([h] * len(frames), frames, outs)), stream)
        for _ in range(args.launches):
            b.replay(stream)
    else:
        for _ in range(args.launches):
            for f, o in zip(frames, outs):
                h.compute(f, o, stream)
    torch.cuda.synchronize()
    print(f"{args.mode}: {args.launches} launches over {len(frames)} frames", flush=True)


if __name__ == "__main__":
    main()
