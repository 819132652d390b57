"""Train the DM-proposal network on the GPU with the project's own kernels.

Training tiles come from fine-bin beam power with injected pulses (synth.power:
noise plus 1-3 pulses in half of the tiles, DM uniform over the grid, S/N 5-50)
turned into DM-time tiles by the library's tile kernel; the network's forward,
loss, backward and Adam steps are the library's.  Writes the flat parameter
vector (float32, include/ddx.h order) to an .npz file.

    python -m paper_1109_3186_amd.train_proposal --tiles 100000 --out paper_1109_3186_amd/proposal_weights.npz
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def make_plan(p, max_block=1 << 15):
    """A plan on the workload's channels and DM grid (its delay tables drive the tiles)."""
    import synth
    from paper_1109_3186_amd import Plan
    fc = synth.chan_freqs(p["f_lo"], p["n_chan"], p["f_s"])
    plan = Plan(p["m_ant"], fc, p["f_s"], p["dump_len"], max_block_samples=max_block, in_dtype="ci8")
    plan.set_dm_trials(synth.dm_grid(p["n_dm"], p["dm_max"]))
    return plan


def he_init(seed):
    """He-normal initial parameters (biases zero), flat in the library's order."""
    import numpy as np

    from paper_1109_3186_amd.proposal import PARAM_SHAPES, flatten
    rng = np.random.Generator(np.random.PCG64(seed))
    params = {}
    for k, shp in PARAM_SHAPES:
        if k.startswith("b"):
            params[k] = np.zeros(shp)
        elif k == "w5":
            params[k] = rng.standard_normal(shp) * np.sqrt(1.0 / shp[0])
        else:
            params[k] = rng.standard_normal(shp) * np.sqrt(2.0 / (shp[1] * shp[2]))
    return flatten(params)


def train(n_tiles, batch, lr, seed, fine=32, log_every=200, out=None, precision="fp16"):
    import numpy as np
    import torch

    import synth
    from paper_1109_3186_amd import Cnn
    dev = torch.device("cuda:0")
    p = synth.c1_params()
    plan = make_plan(p)
    net = Cnn(p["n_dm"], 1024, batch, precision=precision)
    net.set_weights(he_init(seed))
    rng = np.random.Generator(np.random.PCG64(seed))
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    steps = n_tiles // batch
    t0 = time.time()
    hist = []
    for it in range(steps):
        power, labels, _ = synth.power_batch(p, batch, fine, rng, gen, dev)
        tiles = plan.tiles_from_power(power, fine, 1024, 1024)
        net.forward(tiles)
        loss = net.loss(labels.reshape(-1))
        net.backward()
        net.adam(lr=lr)
        if (it + 1) % log_every == 0:
            torch.cuda.synchronize()
            hist.append({"step": it + 1, "loss": float(loss.mean()), "s": round(time.time() - t0, 1)})
            print(json.dumps(hist[-1]), flush=True)
    torch.cuda.synchronize()
    w = net.get_weights()
    if out:
        np.savez(out, params=w, meta=np.array(json.dumps({"tiles": n_tiles, "batch": batch, "lr": lr, "seed": seed,
                                                          "fine": fine, "precision": precision,
                                                          "seconds": time.time() - t0})))
    net.close()
    plan.close()
    return w, hist


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--tiles", type=int, default=100000)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=1114)
    ap.add_argument("--precision", choices=["fp32", "fp16"], default="fp16")
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "proposal_weights.npz"))
    a = ap.parse_args()
    train(a.tiles, a.batch, a.lr, a.seed, out=a.out, precision=a.precision)


if __name__ == "__main__":
    main()
