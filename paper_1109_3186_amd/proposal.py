"""Learned DM proposal: rank the trial DMs of a stream from its DM-time power
tile, and run coherent dedispersion + correlation only on the best-ranked ones.

Steps (all on the GPU through the C ABI): the power tile of the whole stream
(`ddx_power_tile`, the incoherent dedispersion of power beams), the network's
score of every DM row (`ddx_cnn_forward`), then the device top-k of the
scores sets the plan's active DMs (`ddx_select_active_dms`) to the ceil(budget
D) best rows.  Fallback to the full sweep: when more rows than the budget score
above the decision threshold (probability > threshold), the proposal cannot keep
all candidates and the plan runs every DM.
"""
import math

import numpy as np

from .binding import Cnn

# Order of the flat parameter vector (include/ddx.h, ddx_cnn_set_weights).
PARAM_SHAPES = [("W1", (32, 3, 9)), ("b1", (32,)), ("W2", (32, 32, 9)), ("b2", (32,)), ("W3", (32, 32, 9)),
                ("b3", (32,)), ("W4", (32, 32, 9)), ("b4", (32,)), ("w5", (32,)), ("b5", (1,))]


def flatten(params):
    """dict of named arrays -> flat float32 vector in the library's order."""
    return np.concatenate([np.asarray(params[k], dtype=np.float64).reshape(-1) for k, _ in PARAM_SHAPES]).astype(
        np.float32)


def unflatten(flat):
    out, o = {}, 0
    for k, shp in PARAM_SHAPES:
        n = int(np.prod(shp))
        out[k] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def load_weights(path):
    with np.load(path, allow_pickle=False) as z:
        return np.asarray(z["params"], dtype=np.float32)


class Proposal:
    """Tile -> scores -> active-DM mask for one plan."""

    def __init__(self, plan, weights, budget=0.1, threshold=0.5, bin_len=1024, n_bins=1024, precision="fp16"):
        lay = plan.layout()
        self.plan = plan
        self.n_dm = int(lay["n_dm"][0])
        self.k = int(math.ceil(budget * self.n_dm))
        self.threshold = threshold
        self.bin_len, self.n_bins = bin_len, n_bins
        self.net = Cnn(self.n_dm, n_bins, 1, precision=precision)
        self.net.set_weights(weights)
        self.tile = None
        self.scores = None

    def select(self, volts, stream=None):
        """Score the stream's DM rows and set the plan's active DMs (the library
        synchronises `stream` before returning); returns (mask uint8 [D] on the host,
        scores [D] on the device, fallback)."""
        self.tile = self.plan.power_tile(volts, self.bin_len, self.n_bins, out=self.tile, stream=stream)
        self.scores = self.net.forward(self.tile[None], scores=self.scores, stream=stream)
        logit = math.log(self.threshold / (1.0 - self.threshold))
        self.mask, fallback = self.plan.select_active_dms(self.scores, self.k, logit, mask_out=getattr(self, "mask", None),
                                                          stream=stream)
        return self.mask.cpu().numpy(), self.scores, fallback

    def close(self):
        self.net.close()
