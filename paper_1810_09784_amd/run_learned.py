"""Train the tile CNN on the GPU and compare it with the plain selection.

python -m paper_1810_09784_amd.run_learned --out DIR [--pos 10000 --neg-maps 850 --epochs 12]

Writes DIR/tile_cnn.npy (float32 parameters) and DIR/learned.json (training
loss per epoch, thresholds at the target false-alarm probability and the
detection-efficiency curves of both pipelines).  Progress on stderr."""
import argparse
import json
import os
import sys
import time

import numpy as np


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--pos", type=int, default=10000)
    ap.add_argument("--neg-maps", type=int, default=850)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--lr", type=float, default=3e-4)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--noise-maps", type=int, default=5000)
    ap.add_argument("--per-amp", type=int, default=400)
    ap.add_argument("--amps", default="0.3,0.4,0.5,0.7,1.0,1.5,2.0")
    ap.add_argument("--amp-lo", type=float, default=0.25)
    ap.add_argument("--amp-hi", type=float, default=6.0)
    ap.add_argument("--fap", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--weights", default=None, help="skip training, evaluate these parameters")
    ap.add_argument("--checkpoint", default=None,
                    help="training checkpoint (.npz) written after every epoch; an existing one is resumed")
    ap.add_argument("--geometry", default="small", choices=("small", "sweep"),
                    help="small: the n = 5, 500-600 Hz maps; sweep: the full sweep's maps")
    ap.add_argument("--sweep-maps", type=int, default=1250, help="training peakmaps of the sweep geometry")
    ap.add_argument("--sweep-noise", type=int, default=5,
                    help="noise-only sweeps that calibrate the fixed-FAP thresholds (0: none)")
    ap.add_argument("--sweep-inj", type=int, default=200, help="injections of the evaluated sweep")
    ap.add_argument("--sweep-faps", default="0.1,0.03,0.01", help="false-alarm probabilities per map on the sweep")
    a = ap.parse_args()
    import torch
    from . import fh, learn

    def log(*x):
        print(*x, file=sys.stderr, flush=True)

    os.makedirs(a.out, exist_ok=True)
    dev = torch.device("cuda:0")
    net = fh.CNN(max_batch=max(a.batch, 64))
    res = {"config": vars(a)}
    if a.weights:
        net.set_params(np.load(a.weights))
    else:
        rng = np.random.default_rng(a.seed)
        # He-normal conv weights, zero biases, small head
        th = []
        for ci, co in ((1, 16), (16, 32), (32, 64), (64, 64)):
            th += [rng.normal(0, np.sqrt(2.0 / (9 * ci)), co * 9 * ci), np.zeros(co)]
        th += [rng.normal(0, 0.1, 64), np.zeros(1)]
        net.set_params(np.concatenate(th))
        t = time.time()
        if a.geometry == "sweep":
            X, y = learn.build_training_set_sweep(dev, a.sweep_maps, a.seed, amp_lo=a.amp_lo, amp_hi=a.amp_hi,
                                                  log=log)
        else:
            X, y = learn.build_training_set(dev, a.pos, a.neg_maps, a.seed, amp_lo=a.amp_lo, amp_hi=a.amp_hi)
        torch.cuda.synchronize()
        log(f"training set: {X.shape[0]} tiles ({int(y.sum().item())} positive) in {time.time() - t:.1f} s")
        t = time.time()
        hist = learn.train(net, X, y, a.epochs, a.lr, a.batch, a.seed, log=log, checkpoint=a.checkpoint)
        torch.cuda.synchronize()
        dt = time.time() - t
        steps = a.epochs * (X.shape[0] // a.batch)
        flop = steps * a.batch * 3 * 492.4e6
        res["training"] = {"loss": hist, "seconds": dt, "steps": steps, "tiles_per_s": steps * a.batch / dt,
                           "approx_tflops": flop / dt / 1e12}
        p, _ = net.get_params()
        np.save(os.path.join(a.out, "tile_cnn.npy"), p)
        del X, y
    t = time.time()
    if a.geometry == "sweep":
        from . import sweep
        sw = sweep.Sweep(dev, seed=a.seed + 100, n_inj=a.sweep_inj, log=log)
        res["evaluation"] = sweep.evaluate(sw, net)
        if a.sweep_noise > 0:
            faps = [float(x) for x in a.sweep_faps.split(",")]
            res["evaluation"]["at_fap"] = sweep.evaluate_at_fap(dev, net, faps, a.sweep_noise, a.seed + 100, sw=sw,
                                                                log=log)
        sw.destroy()
    else:
        amps = [float(x) for x in a.amps.split(",")]
        res["evaluation"] = learn.evaluate(dev, net, amps, a.noise_maps, a.per_amp, a.seed + 100, a.fap, log=log)
    res["evaluation"]["seconds"] = time.time() - t
    with open(os.path.join(a.out, "learned.json"), "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res["evaluation"]))


if __name__ == "__main__":
    main()
