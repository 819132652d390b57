"""ctypes binding of libddx (include/ddx.h): argument marshalling only.

Every step of the dedispersion/correlation path runs in the HIP library; this
module only converts Python/numpy/torch arguments to C pointers and sizes and
turns status codes into exceptions.  It fails loudly if the library is missing.
"""
import ctypes as ct
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# DDX_LIB_PATH selects another build of the same library (the host-sanitizer
# build of the host-side checks); by default the in-tree libddx.so.
LIB_PATH = os.environ.get("DDX_LIB_PATH") or os.path.join(HERE, "libddx.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ESIZE, EFULL, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
IN_CI8, IN_CF32 = 0, 1
CORR_F32, CORR_F16, CORR_E4M3 = 0, 1, 2
OUT_PACKED, OUT_FULL = 0, 1
FLUSH = 1

_IN = {"ci8": IN_CI8, "cf32": IN_CF32}
_CORR = {"f32": CORR_F32, "f16": CORR_F16, "e4m3": CORR_E4M3}
_OUT = {"packed": OUT_PACKED, "full": OUT_FULL}


class Desc(ct.Structure):
    _fields_ = [
        ("n_ant", ct.c_int32), ("n_chan", ct.c_int32), ("chan_freq_hz", ct.POINTER(ct.c_double)),
        ("samp_rate_hz", ct.c_double), ("sideband", ct.c_int32), ("in_dtype", ct.c_int32),
        ("corr_dtype", ct.c_int32), ("dump_len", ct.c_int32), ("fft_len", ct.POINTER(ct.c_int32)),
        ("k_dm", ct.c_double), ("max_block_samples", ct.c_int64), ("max_device_bytes", ct.c_size_t),
        ("out_mode", ct.c_int32), ("chan_scale", ct.POINTER(ct.c_float)),
        ("wave_units", ct.c_int32), ("dm_group", ct.c_int32), ("compact_records", ct.c_int32),
        ("max_record_pairs", ct.c_int32), ("ring_dumps", ct.c_int64),
        ("dm_classes", ct.c_int32), ("pad", ct.c_int32), ("spectrum_bytes", ct.c_int64),
        ("cost_ps", ct.POINTER(ct.c_double)),
    ]


class Layout(ct.Structure):
    _fields_ = [
        ("n_ant", ct.c_int32), ("n_chan", ct.c_int32), ("n_baselines", ct.c_int32), ("dump_len", ct.c_int32),
        ("out_mode", ct.c_int32), ("corr_dtype", ct.c_int32), ("in_dtype", ct.c_int32), ("sideband", ct.c_int32),
        ("samp_rate_hz", ct.c_double), ("k_dm", ct.c_double),
        ("chan_freq_hz", ct.POINTER(ct.c_double)), ("fft_len", ct.POINTER(ct.c_int32)),
        ("valid", ct.POINTER(ct.c_int32)), ("lead", ct.POINTER(ct.c_int32)), ("n_dm", ct.POINTER(ct.c_int32)),
        ("dm_offset", ct.POINTER(ct.c_int64)), ("dm", ct.POINTER(ct.c_double)),
        ("delay_s", ct.POINTER(ct.c_double)), ("shift", ct.POINTER(ct.c_int64)), ("scale", ct.POINTER(ct.c_float)),
        ("record_pos", ct.POINTER(ct.c_int32)), ("record_pairs", ct.c_int64),
        ("record_elems", ct.c_int64), ("samples_in", ct.c_int64), ("dumps_ready", ct.c_int64),
        ("dumps_fetched", ct.c_int64), ("ring_dumps", ct.c_int64), ("device_bytes", ct.c_size_t),
        ("wave_units", ct.c_int32), ("dm_group", ct.c_int32), ("compact_records", ct.c_int32), ("pad", ct.c_int32),
        ("dump_t0_s", ct.c_double), ("dump_period_s", ct.c_double),
        ("dm_fft_len", ct.POINTER(ct.c_int32)), ("dm_valid", ct.POINTER(ct.c_int32)),
        ("dm_lead", ct.POINTER(ct.c_int32)), ("n_classes", ct.c_int32), ("pad2", ct.c_int32),
    ]


N_KINDS = 5
KIND_NAMES = ["forward", "chirp", "dedisperse", "correlate", "other"]


class Profile(ct.Structure):
    _fields_ = [("launches", ct.c_int64 * N_KINDS), ("time_ms", ct.c_double * N_KINDS),
                ("flops", ct.c_double * N_KINDS), ("bytes", ct.c_double * N_KINDS)]


# Every entry point of include/ddx.h with its argument and result types.
SIGNATURES = {
    "ddx_plan_create": ([ct.POINTER(Desc), ct.POINTER(ct.c_void_p)], ct.c_int),
    "ddx_set_dm_trials": ([ct.c_void_p, ct.c_int32, ct.POINTER(ct.c_double), ct.c_int32], ct.c_int),
    "ddx_set_active_dms": ([ct.c_void_p, ct.c_int32, ct.POINTER(ct.c_uint8)], ct.c_int),
    "ddx_plan_blocking": ([ct.POINTER(Desc), ct.c_int32, ct.POINTER(ct.c_double), ct.c_int32,
                           ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32)], ct.c_int),
    "ddx_get_layout": ([ct.c_void_p, ct.POINTER(Layout)], ct.c_int),
    "ddx_select_active_dms": ([ct.c_void_p, ct.c_int32, ct.c_void_p, ct.c_int32, ct.c_float, ct.c_void_p,
                               ct.POINTER(ct.c_int32), ct.c_void_p], ct.c_int),
    "ddx_dump_times": ([ct.c_void_p, ct.c_int32, ct.c_int32, ct.c_int64, ct.c_int64, ct.c_int32,
                        ct.POINTER(ct.c_double)], ct.c_int),
    "ddx_process_block": ([ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_void_p], ct.c_int),
    "ddx_fetch_visibilities": ([ct.c_void_p, ct.c_void_p, ct.c_size_t, ct.POINTER(ct.c_int64),
                                ct.POINTER(ct.c_int64), ct.c_void_p], ct.c_int),
    "ddx_reset_stream": ([ct.c_void_p], ct.c_int),
    "ddx_set_profiling": ([ct.c_void_p, ct.c_int32], ct.c_int),
    "ddx_get_profile": ([ct.c_void_p, ct.POINTER(Profile)], ct.c_int),
    "ddx_power_tile": ([ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_int32, ct.c_void_p, ct.c_void_p],
                       ct.c_int),
    "ddx_power_tile_from_power": ([ct.c_void_p, ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_int32, ct.c_int32,
                                   ct.c_int32, ct.c_void_p, ct.c_void_p], ct.c_int),
    "ddx_cnn_num_params": ([ct.POINTER(ct.c_int64)], ct.c_int),
    "ddx_cnn_create": ([ct.c_int32, ct.c_int32, ct.c_int32, ct.POINTER(ct.c_void_p)], ct.c_int),
    "ddx_cnn_set_weights": ([ct.c_void_p, ct.POINTER(ct.c_float), ct.c_int64], ct.c_int),
    "ddx_cnn_get_weights": ([ct.c_void_p, ct.POINTER(ct.c_float), ct.c_int64], ct.c_int),
    "ddx_cnn_get_grads": ([ct.c_void_p, ct.POINTER(ct.c_float), ct.c_int64], ct.c_int),
    "ddx_cnn_set_precision": ([ct.c_void_p, ct.c_int32], ct.c_int),
    "ddx_cnn_get_activations": ([ct.c_void_p, ct.c_int32, ct.POINTER(ct.c_float), ct.c_int64], ct.c_int),
    "ddx_cnn_forward": ([ct.c_void_p, ct.c_void_p, ct.c_int32, ct.c_void_p, ct.c_void_p], ct.c_int),
    "ddx_cnn_loss": ([ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p], ct.c_int),
    "ddx_cnn_backward": ([ct.c_void_p, ct.c_void_p], ct.c_int),
    "ddx_cnn_adam": ([ct.c_void_p, ct.c_float, ct.c_float, ct.c_float, ct.c_float, ct.c_void_p], ct.c_int),
    "ddx_cnn_destroy": ([ct.c_void_p], ct.c_int),
    "ddx_cnn_last_error": ([ct.c_void_p], ct.c_char_p),
    "ddx_chirp_create": ([ct.c_int32, ct.c_int32, ct.c_int32, ct.c_int32, ct.c_int64, ct.POINTER(ct.c_void_p)],
                         ct.c_int),
    "ddx_chirp_output_shape": ([ct.c_void_p, ct.c_int64, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int32),
                                ct.POINTER(ct.c_int32)], ct.c_int),
    "ddx_chirp_preintegrate": ([ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_void_p, ct.c_void_p], ct.c_int),
    "ddx_chirp_set_pair_bins": ([ct.c_void_p, ct.POINTER(ct.c_int32)], ct.c_int),
    "ddx_chirp_bank_set_pair_bins": ([ct.c_void_p, ct.POINTER(ct.c_int32)], ct.c_int),
    "ddx_chirp_destroy": ([ct.c_void_p], ct.c_int),
    "ddx_chirp_last_error": ([ct.c_void_p], ct.c_char_p),
    "ddx_chirp_bank_create": ([ct.c_int32, ct.c_int32, ct.c_int32, ct.c_int32, ct.c_int32, ct.c_int64,
                               ct.POINTER(ct.c_void_p)], ct.c_int),
    "ddx_chirp_bank_layout": ([ct.c_void_p, ct.c_int64, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int64),
                               ct.POINTER(ct.c_int64)], ct.c_int),
    "ddx_chirp_bank_run": ([ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_void_p, ct.c_void_p], ct.c_int),
    "ddx_chirp_bank_destroy": ([ct.c_void_p], ct.c_int),
    "ddx_chirp_bank_last_error": ([ct.c_void_p], ct.c_char_p),
    "ddx_image_create": ([ct.c_int32, ct.POINTER(ct.c_double), ct.c_int32, ct.POINTER(ct.c_double), ct.c_double,
                          ct.c_double, ct.c_int32, ct.c_int32, ct.c_int32, ct.c_int32, ct.POINTER(ct.c_void_p)],
                         ct.c_int),
    "ddx_image_output_count": ([ct.c_void_p, ct.c_int64, ct.c_int32, ct.POINTER(ct.c_int64)], ct.c_int),
    "ddx_image_run": ([ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int64, ct.c_int32, ct.c_void_p, ct.c_void_p,
                       ct.c_void_p], ct.c_int),
    "ddx_image_destroy": ([ct.c_void_p], ct.c_int),
    "ddx_image_last_error": ([ct.c_void_p], ct.c_char_p),
    "ddx_power_beam": ([ct.c_void_p, ct.c_int32, ct.c_int32, ct.c_int64, ct.c_int32, ct.c_void_p, ct.c_void_p],
                       ct.c_int),
    "ddx_incoherent_delays": ([ct.c_int32, ct.POINTER(ct.c_double), ct.c_double, ct.c_int32,
                               ct.POINTER(ct.c_double), ct.c_double, ct.POINTER(ct.c_int32)], ct.c_int),
    "ddx_incoherent_dedisperse": ([ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_void_p, ct.c_int32, ct.c_void_p,
                                   ct.c_int64, ct.c_void_p], ct.c_int),
    "ddx_tree_dedisperse": ([ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_void_p, ct.c_void_p, ct.c_void_p], ct.c_int),
    "ddx_tree_dedisperse_static": ([ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_void_p, ct.c_void_p], ct.c_int),
    "ddx_chimg_sampling_blocks": ([ct.c_double, ct.c_int32, ct.c_double], ct.c_int),
    "ddx_chimg_trajectories_ext": ([ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_int32, ct.c_int32, ct.c_void_p,
                                    ct.c_void_p, ct.c_void_p, ct.c_int32, ct.c_int32, ct.c_void_p, ct.c_void_p],
                                   ct.c_int),
    "ddx_chimg_cells_2d": ([ct.c_int32, ct.POINTER(ct.c_double), ct.c_double, ct.c_int32, ct.POINTER(ct.c_int32),
                            ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32),
                            ct.POINTER(ct.c_int32)], ct.c_int),
    "ddx_chimg_preintegrate_2d": ([ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_int32, ct.c_int32, ct.c_int32,
                                   ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p], ct.c_int),
    "ddx_chimg_trajectories_2d": ([ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_int32, ct.c_int32, ct.c_void_p,
                                   ct.c_void_p, ct.c_void_p, ct.c_int32, ct.c_int32, ct.c_void_p, ct.c_void_p,
                                   ct.c_void_p, ct.c_void_p], ct.c_int),
    "ddx_chimg_preintegrate": ([ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_int32, ct.c_int32, ct.c_int32, ct.c_void_p,
                                ct.c_void_p], ct.c_int),
    "ddx_chimg_trajectories": ([ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_int32, ct.c_int32, ct.c_void_p, ct.c_void_p,
                                ct.c_int32, ct.c_void_p, ct.c_void_p], ct.c_int),
    "ddx_chimg_gradient_sums": ([ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_int32, ct.c_int32, ct.c_void_p,
                                 ct.c_int32, ct.c_void_p, ct.c_int32, ct.c_void_p, ct.c_void_p], ct.c_int),
    "ddx_chimg_cells": ([ct.c_int32, ct.POINTER(ct.c_double), ct.c_double, ct.c_int32, ct.POINTER(ct.c_int32),
                         ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32)], ct.c_int),
    "ddx_chimg_preintegrate_cells": ([ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_int32, ct.c_int32, ct.c_int32,
                                      ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p], ct.c_int),
    "ddx_plan_destroy": ([ct.c_void_p], ct.c_int),
    "ddx_strerror": ([ct.c_int], ct.c_char_p),
    "ddx_last_error": ([ct.c_void_p], ct.c_char_p),
}

_lib = None


def lib():
    """Load libddx.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("%s not built: run __graft_entry__.build() (or python -m paper_1109_3186_amd.build)" % LIB_PATH)
        L = ct.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


class DdxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (lib().ddx_strerror(status).decode(), status, msg))
        self.status = status


def _stream_handle(stream):
    if stream is None:
        import torch
        return ct.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ct.c_void_p(stream)
    return ct.c_void_p(stream.cuda_stream)


class Plan:
    """One ddx plan (see include/ddx.h for the semantics of every call)."""

    def __init__(self, n_ant, chan_freqs, samp_rate, dump_len, max_block_samples, *, sideband=1, in_dtype="ci8",
                 corr_dtype="f32", fft_len=None, k_dm=0.0, max_device_bytes=0, out_mode="packed", chan_scale=None,
                 wave_units=0, dm_group=0, compact_records=False, max_record_pairs=0, ring_dumps=0,
                 dm_classes="auto", spectrum_bytes=0, cost_ps=None):
        L = lib()
        fc = np.ascontiguousarray(chan_freqs, dtype=np.float64)
        self._fc = fc
        d = Desc()
        d.n_ant = n_ant
        d.n_chan = len(fc)
        d.chan_freq_hz = fc.ctypes.data_as(ct.POINTER(ct.c_double))
        d.samp_rate_hz = samp_rate
        d.sideband = sideband
        d.in_dtype = _IN[in_dtype]
        d.corr_dtype = _CORR[corr_dtype]
        d.dump_len = dump_len
        if fft_len is not None:
            self._fft = np.ascontiguousarray(np.broadcast_to(fft_len, fc.shape), dtype=np.int32)
            d.fft_len = self._fft.ctypes.data_as(ct.POINTER(ct.c_int32))
        d.k_dm = k_dm
        d.max_block_samples = int(max_block_samples)
        d.max_device_bytes = int(max_device_bytes)
        d.out_mode = _OUT[out_mode]
        if chan_scale is not None:
            self._scale = np.ascontiguousarray(np.broadcast_to(chan_scale, fc.shape), dtype=np.float32)
            d.chan_scale = self._scale.ctypes.data_as(ct.POINTER(ct.c_float))
        d.wave_units = int(wave_units)
        d.dm_group = int(dm_group)
        d.compact_records = 1 if compact_records else 0
        d.max_record_pairs = int(max_record_pairs)
        d.ring_dumps = int(ring_dumps)
        # "auto": each channel's DMs in blocking classes by the cost model; "single": one per channel
        d.dm_classes = {"auto": 0, "single": 1}[dm_classes]
        d.spectrum_bytes = int(spectrum_bytes)
        if cost_ps is not None:  # [2][11] ps per point (inverse, forward) for N = 2^8 .. 2^18
            self._cost = np.ascontiguousarray(cost_ps, dtype=np.float64).reshape(22)
            d.cost_ps = self._cost.ctypes.data_as(ct.POINTER(ct.c_double))
        h = ct.c_void_p()
        rc = L.ddx_plan_create(ct.byref(d), ct.byref(h))
        if rc != OK:
            raise DdxError(rc, "ddx_plan_create")
        self._h = h
        self.n_ant = n_ant
        self.in_dtype = in_dtype
        self.max_block = int(max_block_samples)

    def _check(self, rc, what):
        if rc != OK:
            raise DdxError(rc, "%s: %s" % (what, lib().ddx_last_error(self._h).decode()))

    def set_dm_trials(self, dms, chan=-1):
        a = np.ascontiguousarray(dms, dtype=np.float64)
        self._check(lib().ddx_set_dm_trials(self._h, chan, a.ctypes.data_as(ct.POINTER(ct.c_double)), len(a)),
                    "ddx_set_dm_trials")

    def set_active_dms(self, mask, chan=-1):
        if mask is None:
            ptr = None
        else:
            m = np.ascontiguousarray(mask, dtype=np.uint8)
            ptr = m.ctypes.data_as(ct.POINTER(ct.c_uint8))
        self._check(lib().ddx_set_active_dms(self._h, chan, ptr), "ddx_set_active_dms")

    def select_active_dms(self, scores, k, logit_threshold=0.0, chan=-1, mask_out=None, stream=None):
        """Device top-k of per-DM logits (ddx_select_active_dms): activates the k best
        DMs, or all of them when more than k logits exceed logit_threshold.  scores:
        device float32 [D].  Returns (mask: device uint8 [D], fallback: bool)."""
        import torch
        if scores.dtype != torch.float32 or not scores.is_cuda or not scores.is_contiguous():
            raise ValueError("scores must be a contiguous float32 device tensor")
        if mask_out is None:
            mask_out = torch.empty(scores.numel(), dtype=torch.uint8, device=scores.device)
        fb = ct.c_int32(0)
        self._check(lib().ddx_select_active_dms(self._h, chan, ct.c_void_p(scores.data_ptr()), int(k),
                                                float(logit_threshold), ct.c_void_p(mask_out.data_ptr()),
                                                ct.byref(fb), _stream_handle(stream)), "ddx_select_active_dms")
        return mask_out, bool(fb.value)

    def layout(self):
        lay = Layout()
        self._check(lib().ddx_get_layout(self._h, ct.byref(lay)), "ddx_get_layout")
        C = lay.n_chan

        def arr(ptr, n, dt):
            return np.ctypeslib.as_array(ptr, shape=(n,)).astype(dt).copy()

        off = arr(lay.dm_offset, C + 1, np.int64)
        nd = int(off[-1])
        return {
            "n_ant": lay.n_ant, "n_chan": C, "n_baselines": lay.n_baselines, "dump_len": lay.dump_len,
            "out_mode": lay.out_mode, "corr_dtype": lay.corr_dtype, "in_dtype": lay.in_dtype,
            "sideband": lay.sideband, "samp_rate_hz": lay.samp_rate_hz, "k_dm": lay.k_dm,
            "chan_freq_hz": arr(lay.chan_freq_hz, C, np.float64), "fft_len": arr(lay.fft_len, C, np.int64),
            "valid": arr(lay.valid, C, np.int64), "lead": arr(lay.lead, C, np.int64),
            "n_dm": arr(lay.n_dm, C, np.int64), "dm_offset": off, "dm": arr(lay.dm, nd, np.float64),
            "delay_s": arr(lay.delay_s, nd, np.float64), "shift": arr(lay.shift, nd, np.int64),
            "scale": arr(lay.scale, C, np.float32), "record_pos": arr(lay.record_pos, nd, np.int64),
            "record_pairs": lay.record_pairs, "record_elems": lay.record_elems,
            "samples_in": lay.samples_in, "dumps_ready": lay.dumps_ready, "dumps_fetched": lay.dumps_fetched,
            "ring_dumps": lay.ring_dumps, "device_bytes": lay.device_bytes, "wave_units": lay.wave_units,
            "dm_group": lay.dm_group, "compact_records": lay.compact_records,
            "dump_t0_s": lay.dump_t0_s, "dump_period_s": lay.dump_period_s,
            "dm_fft_len": arr(lay.dm_fft_len, nd, np.int64), "dm_valid": arr(lay.dm_valid, nd, np.int64),
            "dm_lead": arr(lay.dm_lead, nd, np.int64), "n_classes": lay.n_classes,
        }

    def dump_times(self, chan, dm_index, first_dump, n_dumps, refer_infinite=False):
        """FP64 times (s) of dumps first_dump .. first_dump + n_dumps - 1 (ddx_dump_times)."""
        out = np.zeros(max(int(n_dumps), 0), dtype=np.float64)
        self._check(lib().ddx_dump_times(self._h, chan, dm_index, first_dump, n_dumps, int(bool(refer_infinite)),
                                         out.ctypes.data_as(ct.POINTER(ct.c_double))), "ddx_dump_times")
        return out

    def process_block(self, volts, flush=False, stream=None):
        """volts: torch device tensor, int8 [C, M, 2n] (ci8) or complex64 [C, M, n] (cf32), contiguous."""
        if volts is None:
            n, ptr = 0, None
        else:
            if not volts.is_cuda or not volts.is_contiguous():
                raise ValueError("volts must be a contiguous device tensor")
            import torch
            if self.in_dtype == "ci8":
                if volts.dtype != torch.int8:
                    raise ValueError("ci8 plan needs an int8 tensor [C, M, 2n]")
                n = volts.shape[-1] // 2
            else:
                if volts.dtype != torch.complex64:
                    raise ValueError("cf32 plan needs a complex64 tensor [C, M, n]")
                n = volts.shape[-1]
            ptr = ct.c_void_p(volts.data_ptr())
        rc = lib().ddx_process_block(self._h, ptr, int(n), FLUSH if flush else 0, _stream_handle(stream))
        self._check(rc, "ddx_process_block")

    def fetch(self, out=None, stream=None):
        """Return (first_dump, n_dumps, tensor [n_dumps, record_elems] complex64 on the device)."""
        import torch
        first, nd = ct.c_int64(), ct.c_int64()
        st = _stream_handle(stream)
        rc = lib().ddx_fetch_visibilities(self._h, None, 0, ct.byref(first), ct.byref(nd), st)
        if rc == OK and nd.value == 0:
            return first.value, 0, None
        if rc not in (OK, ESIZE):
            self._check(rc, "ddx_fetch_visibilities")
        need = nd.value
        rec = self.layout()["record_elems"]
        if out is None:
            out = torch.empty((need, rec), dtype=torch.complex64, device="cuda")
        elif out.numel() < need * rec or out.dtype != torch.complex64 or not out.is_contiguous():
            raise ValueError("output tensor too small or not contiguous complex64")
        rc = lib().ddx_fetch_visibilities(self._h, ct.c_void_p(out.data_ptr()), out.numel() * 8, ct.byref(first),
                                          ct.byref(nd), st)
        self._check(rc, "ddx_fetch_visibilities")
        return first.value, nd.value, out.view(-1)[: need * rec].view(need, rec)

    def reset_stream(self):
        self._check(lib().ddx_reset_stream(self._h), "ddx_reset_stream")

    def set_profiling(self, on):
        self._check(lib().ddx_set_profiling(self._h, 1 if on else 0), "ddx_set_profiling")

    def profile(self):
        pr = Profile()
        self._check(lib().ddx_get_profile(self._h, ct.byref(pr)), "ddx_get_profile")
        return {KIND_NAMES[k]: {"launches": pr.launches[k], "time_ms": pr.time_ms[k], "flops": pr.flops[k],
                                "bytes": pr.bytes[k]} for k in range(N_KINDS)}

    def power_tile(self, volts, bin_len, n_bins, out=None, stream=None):
        """DM-time tile [D, n_bins] of one whole stream (device tensor as for process_block)."""
        import torch
        n = volts.shape[-1] // 2 if self.in_dtype == "ci8" else volts.shape[-1]
        d = int(self.layout()["n_dm"][0])
        if out is None:
            out = torch.empty((d, n_bins), dtype=torch.float32, device=volts.device)
        self._check(lib().ddx_power_tile(self._h, ct.c_void_p(volts.data_ptr()), int(n), bin_len, n_bins,
                                         ct.c_void_p(out.data_ptr()), _stream_handle(stream)), "ddx_power_tile")
        return out

    def tiles_from_power(self, power, fine, bin_len, n_bins, out=None, stream=None):
        """Tiles [T, D, n_bins] from fine-bin beam power [T, C, U] (device float32 tensor)."""
        import torch
        t, c, u = power.shape
        d = int(self.layout()["n_dm"][0])
        if out is None:
            out = torch.empty((t, d, n_bins), dtype=torch.float32, device=power.device)
        self._check(lib().ddx_power_tile_from_power(self._h, ct.c_void_p(power.data_ptr()), t, int(u), fine, bin_len,
                                                    n_bins, ct.c_void_p(out.data_ptr()), _stream_handle(stream)),
                    "ddx_power_tile_from_power")
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().ddx_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Cnn:
    """The DM-proposal network of include/ddx.h (ddx_cnn_*)."""

    PRECISIONS = {"fp32": 0, "fp16": 1}

    def __init__(self, n_dm, n_bins, max_tiles, precision="fp32"):
        L = lib()
        n = ct.c_int64()
        L.ddx_cnn_num_params(ct.byref(n))
        self.n_params = n.value
        h = ct.c_void_p()
        rc = L.ddx_cnn_create(n_dm, n_bins, max_tiles, ct.byref(h))
        if rc != OK:
            raise DdxError(rc, "ddx_cnn_create")
        self._h = h
        self.n_dm, self.n_bins, self.max_tiles = n_dm, n_bins, max_tiles
        self.set_precision(precision)

    def set_precision(self, precision):
        """'fp32' (vector units) or 'fp16' (binary16 operands on the matrix cores)."""
        if precision not in self.PRECISIONS:
            raise ValueError("precision must be one of %s" % sorted(self.PRECISIONS))
        self._check(lib().ddx_cnn_set_precision(self._h, self.PRECISIONS[precision]), "ddx_cnn_set_precision")
        self.precision = precision

    def _check(self, rc, what):
        if rc != OK:
            raise DdxError(rc, "%s: %s" % (what, lib().ddx_cnn_last_error(self._h).decode()))

    def set_weights(self, flat):
        a = np.ascontiguousarray(flat, dtype=np.float32)
        self._check(lib().ddx_cnn_set_weights(self._h, a.ctypes.data_as(ct.POINTER(ct.c_float)), a.size),
                    "ddx_cnn_set_weights")

    def get_weights(self):
        a = np.empty(self.n_params, dtype=np.float32)
        self._check(lib().ddx_cnn_get_weights(self._h, a.ctypes.data_as(ct.POINTER(ct.c_float)), a.size),
                    "ddx_cnn_get_weights")
        return a

    def get_grads(self):
        a = np.empty(self.n_params, dtype=np.float32)
        self._check(lib().ddx_cnn_get_grads(self._h, a.ctypes.data_as(ct.POINTER(ct.c_float)), a.size),
                    "ddx_cnn_get_grads")
        return a

    def get_activations(self, layer, rows):
        """Layer 1..4's activations of the last forward pass, float32 [rows, 32, n_bins >> (layer - 1)]."""
        a = np.empty((rows, 32, self.n_bins >> (layer - 1)), dtype=np.float32)
        self._check(lib().ddx_cnn_get_activations(self._h, layer, a.ctypes.data_as(ct.POINTER(ct.c_float)), a.size),
                    "ddx_cnn_get_activations")
        return a

    def forward(self, tiles, scores=None, stream=None):
        """tiles: device float32 [T, n_dm, n_bins] (kept alive until backward); returns scores [T * n_dm]."""
        import torch
        t = tiles.shape[0]
        if scores is None:
            scores = torch.empty(t * self.n_dm, dtype=torch.float32, device=tiles.device)
        self._check(lib().ddx_cnn_forward(self._h, ct.c_void_p(tiles.data_ptr()), t, ct.c_void_p(scores.data_ptr()),
                                          _stream_handle(stream)), "ddx_cnn_forward")
        # the library reads both again in loss/backward: keep them alive until the next forward
        self._tiles, self._scores = tiles, scores
        return scores

    def loss(self, labels, loss_rows=None, stream=None):
        import torch
        if loss_rows is None:
            loss_rows = torch.empty_like(labels)
        self._check(lib().ddx_cnn_loss(self._h, ct.c_void_p(labels.data_ptr()), ct.c_void_p(loss_rows.data_ptr()),
                                       _stream_handle(stream)), "ddx_cnn_loss")
        self._labels = labels
        return loss_rows

    def backward(self, stream=None):
        self._check(lib().ddx_cnn_backward(self._h, _stream_handle(stream)), "ddx_cnn_backward")

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        self._check(lib().ddx_cnn_adam(self._h, lr, beta1, beta2, eps, _stream_handle(stream)), "ddx_cnn_adam")

    def close(self):
        if getattr(self, "_h", None):
            lib().ddx_cnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Chirp:
    """The Chirpolator pre-integrator of include/ddx.h (ddx_chirp_*): for every
    antenna pair p < q, bins -kmax..kmax of the sliding DFT of length N, sampled
    every L samples, of the mixed product s_p s_q^*."""

    def __init__(self, n_ant, fft_n, block_len, kmax, max_samples):
        h = ct.c_void_p()
        rc = lib().ddx_chirp_create(n_ant, fft_n, block_len, kmax, max_samples, ct.byref(h))
        if rc != OK:
            raise DdxError(rc, "ddx_chirp_create")
        self._h = h
        self.n_ant, self.fft_n, self.block_len, self.kmax, self.max_samples = n_ant, fft_n, block_len, kmax, max_samples

    def _check(self, rc, what):
        if rc != OK:
            raise DdxError(rc, "%s: %s" % (what, lib().ddx_chirp_last_error(self._h).decode()))

    def set_pair_bins(self, kmax_pair=None):
        """Per-pair bin budgets (row-major pair order), None = kmax for every pair."""
        if kmax_pair is None:
            self._check(lib().ddx_chirp_set_pair_bins(self._h, None), "ddx_chirp_set_pair_bins")
            return
        a = np.ascontiguousarray(kmax_pair, dtype=np.int32)
        self._check(lib().ddx_chirp_set_pair_bins(self._h, a.ctypes.data_as(ct.POINTER(ct.c_int32))),
                    "ddx_chirp_set_pair_bins")

    def output_shape(self, n):
        w, p, b = ct.c_int64(), ct.c_int32(), ct.c_int32()
        self._check(lib().ddx_chirp_output_shape(self._h, int(n), ct.byref(w), ct.byref(p), ct.byref(b)),
                    "ddx_chirp_output_shape")
        return w.value, p.value, b.value

    def preintegrate(self, volts, out=None, stream=None):
        """volts: device complex64 [M, n]; returns device complex64 [windows, pairs, bins]."""
        import torch
        if volts.dtype != torch.complex64 or volts.dim() != 2 or volts.shape[0] != self.n_ant:
            raise DdxError(EINVAL, "volts must be complex64 [%d, n]" % self.n_ant)
        volts = volts.contiguous()
        n = volts.shape[1]
        shape = self.output_shape(n)
        if out is None:
            out = torch.empty(shape, dtype=torch.complex64, device=volts.device)
        elif tuple(out.shape) != shape or out.dtype != torch.complex64 or not out.is_contiguous():
            raise DdxError(EINVAL, "out must be contiguous complex64 %s" % (shape,))
        self._check(lib().ddx_chirp_preintegrate(self._h, ct.c_void_p(volts.data_ptr()), n,
                                                 ct.c_void_p(out.data_ptr()), _stream_handle(stream)),
                    "ddx_chirp_preintegrate")
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().ddx_chirp_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ChirpBank:
    """The bank of pre-integrators over window lengths n0 d, d = 1..n_len, with the
    DFT factorisation of include/ddx.h (ddx_chirp_bank_*)."""

    def __init__(self, n_ant, n0, n_len, block_len, kmax, max_samples):
        h = ct.c_void_p()
        rc = lib().ddx_chirp_bank_create(n_ant, n0, n_len, block_len, kmax, max_samples, ct.byref(h))
        if rc != OK:
            raise DdxError(rc, "ddx_chirp_bank_create")
        self._h = h
        self.n_ant, self.n0, self.n_len, self.block_len, self.kmax = n_ant, n0, n_len, block_len, kmax

    def _check(self, rc, what):
        if rc != OK:
            raise DdxError(rc, "%s: %s" % (what, lib().ddx_chirp_bank_last_error(self._h).decode()))

    def set_pair_bins(self, kmax_pair=None):
        """Per-pair bin budgets for every length (row-major pair order), None = kmax."""
        if kmax_pair is None:
            self._check(lib().ddx_chirp_bank_set_pair_bins(self._h, None), "ddx_chirp_bank_set_pair_bins")
            return
        a = np.ascontiguousarray(kmax_pair, dtype=np.int32)
        self._check(lib().ddx_chirp_bank_set_pair_bins(self._h, a.ctypes.data_as(ct.POINTER(ct.c_int32))),
                    "ddx_chirp_bank_set_pair_bins")

    def layout(self, n):
        w = (ct.c_int64 * self.n_len)()
        o = (ct.c_int64 * self.n_len)()
        t = ct.c_int64()
        self._check(lib().ddx_chirp_bank_layout(self._h, int(n), w, o, ct.byref(t)), "ddx_chirp_bank_layout")
        return list(w), list(o), t.value

    def run(self, volts, out=None, stream=None):
        """volts: device complex64 [M, n]; returns a list of device views [windows_d, pairs, bins], d = 1..n_len."""
        import torch
        if volts.dtype != torch.complex64 or volts.dim() != 2 or volts.shape[0] != self.n_ant:
            raise DdxError(EINVAL, "volts must be complex64 [%d, n]" % self.n_ant)
        volts = volts.contiguous()
        n = volts.shape[1]
        wins, offs, total = self.layout(n)
        if out is None:
            out = torch.empty(max(total, 1), dtype=torch.complex64, device=volts.device)
        self._check(lib().ddx_chirp_bank_run(self._h, ct.c_void_p(volts.data_ptr()), n, ct.c_void_p(out.data_ptr()),
                                             _stream_handle(stream)), "ddx_chirp_bank_run")
        pairs, bins = self.n_ant * (self.n_ant - 1) // 2, 2 * self.kmax + 1
        return [out[o:o + w * pairs * bins].view(w, pairs, bins) for w, o in zip(wins, offs)]

    def close(self):
        if getattr(self, "_h", None):
            lib().ddx_chirp_bank_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Image:
    """The post-integrator detection image of include/ddx.h (ddx_image_*): P and
    E = |P|^2 per window and direction from the pre-integrator's bins."""

    def __init__(self, ant_xyz, pix_lm, fdot, samp_rate, fft_n, block_len, kmax, half_width):
        ant = np.ascontiguousarray(ant_xyz, dtype=np.float64)
        pix = np.ascontiguousarray(pix_lm, dtype=np.float64)
        if ant.ndim != 2 or ant.shape[1] != 3 or pix.ndim != 2 or pix.shape[1] != 2:
            raise DdxError(EINVAL, "ant_xyz must be [M, 3] and pix_lm [n_pix, 2]")
        dp = ct.POINTER(ct.c_double)
        h = ct.c_void_p()
        rc = lib().ddx_image_create(ant.shape[0], ant.ctypes.data_as(dp), pix.shape[0], pix.ctypes.data_as(dp),
                                    float(fdot), float(samp_rate), fft_n, block_len, kmax, half_width, ct.byref(h))
        if rc != OK:
            raise DdxError(rc, "ddx_image_create")
        self._h = h
        self.n_ant, self.n_pix, self.kmax = ant.shape[0], pix.shape[0], kmax

    def _check(self, rc, what):
        if rc != OK:
            raise DdxError(rc, "%s: %s" % (what, lib().ddx_image_last_error(self._h).decode()))

    def output_count(self, n_rows, w_step=1):
        n = ct.c_int64()
        self._check(lib().ddx_image_output_count(self._h, int(n_rows), int(w_step), ct.byref(n)),
                    "ddx_image_output_count")
        return n.value

    def run(self, bins, first_window=0, w_step=1, want_p=True, want_e=True, stream=None):
        """bins: device complex64 [rows, pairs, 2 kmax + 1] (pre-integrator windows
        first_window ..); returns (P complex64 [images, n_pix] or None, E float32 or None)."""
        import torch
        pairs = self.n_ant * (self.n_ant - 1) // 2
        if bins.dtype != torch.complex64 or bins.dim() != 3 or tuple(bins.shape[1:]) != (pairs, 2 * self.kmax + 1):
            raise DdxError(EINVAL, "bins must be complex64 [rows, %d, %d]" % (pairs, 2 * self.kmax + 1))
        bins = bins.contiguous()
        n_img = self.output_count(bins.shape[0], w_step)
        p = torch.empty((n_img, self.n_pix), dtype=torch.complex64, device=bins.device) if want_p else None
        e = torch.empty((n_img, self.n_pix), dtype=torch.float32, device=bins.device) if want_e else None
        self._check(lib().ddx_image_run(self._h, ct.c_void_p(bins.data_ptr()), bins.shape[0], int(first_window),
                                        int(w_step), ct.c_void_p(p.data_ptr() if p is not None else None),
                                        ct.c_void_p(e.data_ptr() if e is not None else None),
                                        _stream_handle(stream)), "ddx_image_run")
        return p, e

    def close(self):
        if getattr(self, "_h", None):
            lib().ddx_image_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def layout_blockings(lay):
    """Per channel, the list of its DMs' blockings ({fft_len, valid, lead}, each that
    of the DM's class) from a Plan.layout() dict."""
    off = lay["dm_offset"]
    return [[{"fft_len": int(lay["dm_fft_len"][k]), "valid": int(lay["dm_valid"][k]), "lead": int(lay["dm_lead"][k])}
             for k in range(off[c], off[c + 1])] for c in range(lay["n_chan"])]


def plan_blocking(chan_freqs, samp_rate, dump_len, dms, chan=0, fft_len=None, k_dm=0.0, dm_classes="auto",
                  cost_ps=None):
    """Per-DM overlap-save blocking a plan would choose for channel chan, on the host
    (ddx_plan_blocking).  Returns (fft_len, valid, lead) int arrays of len(dms) and
    the number of classes."""
    fc = np.ascontiguousarray(chan_freqs, dtype=np.float64)
    d = Desc()
    d.n_ant = 1
    d.n_chan = len(fc)
    d.chan_freq_hz = fc.ctypes.data_as(ct.POINTER(ct.c_double))
    d.samp_rate_hz = samp_rate
    d.sideband = 1
    d.dump_len = dump_len
    d.k_dm = k_dm
    d.max_block_samples = 1
    if fft_len is not None:
        fl = np.ascontiguousarray(np.broadcast_to(fft_len, fc.shape), dtype=np.int32)
        d.fft_len = fl.ctypes.data_as(ct.POINTER(ct.c_int32))
    d.dm_classes = {"auto": 0, "single": 1}[dm_classes]
    if cost_ps is not None:
        cost = np.ascontiguousarray(cost_ps, dtype=np.float64).reshape(22)
        d.cost_ps = cost.ctypes.data_as(ct.POINTER(ct.c_double))
    a = np.ascontiguousarray(dms, dtype=np.float64)
    n, v, l = (np.zeros(len(a), dtype=np.int32) for _ in range(3))
    p32 = ct.POINTER(ct.c_int32)
    rc = lib().ddx_plan_blocking(ct.byref(d), chan, a.ctypes.data_as(ct.POINTER(ct.c_double)), len(a),
                                 n.ctypes.data_as(p32), v.ctypes.data_as(p32), l.ctypes.data_as(p32))
    if rc < 0:
        raise DdxError(rc, "ddx_plan_blocking")
    return n.astype(np.int64), v.astype(np.int64), l.astype(np.int64), rc


def incoherent_delays(chan_freq_hz, t_samp_s, dms, k_dm=4.148808e15):
    """Dispersion delays in samples relative to the highest channel, int32 [C, D]."""
    f = np.ascontiguousarray(chan_freq_hz, dtype=np.float64)
    d = np.ascontiguousarray(dms, dtype=np.float64)
    out = np.empty((f.size, d.size), dtype=np.int32)
    dp = ct.POINTER(ct.c_double)
    rc = lib().ddx_incoherent_delays(f.size, f.ctypes.data_as(dp), float(t_samp_s), d.size, d.ctypes.data_as(dp),
                                     float(k_dm), out.ctypes.data_as(ct.POINTER(ct.c_int32)))
    if rc != OK:
        raise DdxError(rc, "ddx_incoherent_delays")
    return out


def power_beam(volts, n_int, stream=None):
    """volts: device complex64 [C, M, S]; returns device float32 [C, S // n_int]."""
    import torch
    if volts.dtype != torch.complex64 or volts.dim() != 3:
        raise DdxError(EINVAL, "volts must be complex64 [C, M, S]")
    volts = volts.contiguous()
    C, M, S = volts.shape
    out = torch.empty((C, S // n_int), dtype=torch.float32, device=volts.device)
    rc = lib().ddx_power_beam(ct.c_void_p(volts.data_ptr()), C, M, S, int(n_int), ct.c_void_p(out.data_ptr()),
                              _stream_handle(stream))
    if rc != OK:
        raise DdxError(rc, "ddx_power_beam")
    return out


def incoherent_dedisperse(power, delays, n_out, stream=None):
    """power: device float32 [C, T]; delays: device int32 [C, D]; returns [D, n_out]."""
    import torch
    if power.dtype != torch.float32 or power.dim() != 2 or delays.dtype != torch.int32 or \
            tuple(delays.shape[:1]) != (power.shape[0],):
        raise DdxError(EINVAL, "power must be float32 [C, T] and delays int32 [C, D]")
    power, delays = power.contiguous(), delays.contiguous()
    out = torch.empty((delays.shape[1], int(n_out)), dtype=torch.float32, device=power.device)
    rc = lib().ddx_incoherent_dedisperse(ct.c_void_p(power.data_ptr()), power.shape[0], power.shape[1],
                                         ct.c_void_p(delays.data_ptr()), delays.shape[1],
                                         ct.c_void_p(out.data_ptr()), int(n_out), _stream_handle(stream))
    if rc != OK:
        raise DdxError(rc, "ddx_incoherent_dedisperse")
    return out


def tree_dedisperse(power, out=None, work=None, stream=None):
    """The tree method on device float32 [C, T] (C a power of two); returns [C, T]."""
    import torch
    if power.dtype != torch.float32 or power.dim() != 2:
        raise DdxError(EINVAL, "power must be float32 [C, T]")
    power = power.contiguous()
    if out is None:
        out = torch.empty_like(power)
    if work is None:
        work = torch.empty_like(power)
    rc = lib().ddx_tree_dedisperse(ct.c_void_p(power.data_ptr()), power.shape[0], power.shape[1],
                                   ct.c_void_p(out.data_ptr()), ct.c_void_p(work.data_ptr()),
                                   _stream_handle(stream))
    if rc != OK:
        raise DdxError(rc, "ddx_tree_dedisperse")
    return out


TREE_STATIC_MAX = 16 * 1024 * 1024


def tree_dedisperse_static(power, out, stream=None):
    """The tree method with the library's static workspace (no allocation by the
    library or here): device float32 power [C, T] and out [C, T], C T <= TREE_STATIC_MAX."""
    import torch
    if power.dtype != torch.float32 or power.dim() != 2 or not power.is_contiguous():
        raise DdxError(EINVAL, "power must be contiguous float32 [C, T]")
    if out.shape != power.shape or out.dtype != torch.float32 or not out.is_contiguous():
        raise DdxError(EINVAL, "out must be contiguous float32 of power's shape")
    rc = lib().ddx_tree_dedisperse_static(ct.c_void_p(power.data_ptr()), power.shape[0], power.shape[1],
                                          ct.c_void_p(out.data_ptr()), _stream_handle(stream))
    if rc != OK:
        raise DdxError(rc, "ddx_tree_dedisperse_static")
    return out


def chimg_preintegrate(volts, block_len, n_s, natural=True, stream=None):
    """The Chimageator pre-integrator on a uniform linear array: volts device
    complex64 [M, n]; returns device complex64 Y [n_s, n // block_len] (bin-major)."""
    import torch
    if volts.dtype != torch.complex64 or volts.dim() != 2:
        raise DdxError(EINVAL, "volts must be complex64 [M, n]")
    volts = volts.contiguous()
    M, n = volts.shape
    y = torch.empty((n_s, n // block_len), dtype=torch.complex64, device=volts.device)
    rc = lib().ddx_chimg_preintegrate(ct.c_void_p(volts.data_ptr()), M, n, int(block_len), int(n_s),
                                      1 if natural else 0, ct.c_void_p(y.data_ptr()), _stream_handle(stream))
    if rc != OK:
        raise DdxError(rc, "ddx_chimg_preintegrate")
    return y


def chimg_trajectories(y, n_ant, block_len, k_end, t_blocks, stream=None):
    """Trajectory sums P [trials, blocks] (complex64, device) for trials (k_end[i],
    t_blocks[i]) over the pre-integrator output y [n_s, blocks]."""
    import torch
    if y.dtype != torch.complex64 or y.dim() != 2:
        raise DdxError(EINVAL, "y must be complex64 [n_s, blocks]")
    y = y.contiguous()
    ke = torch.as_tensor(np.asarray(k_end, dtype=np.float64), device=y.device)
    tb = torch.as_tensor(np.asarray(t_blocks, dtype=np.int32), device=y.device)
    p = torch.empty((ke.numel(), y.shape[1]), dtype=torch.complex64, device=y.device)
    rc = lib().ddx_chimg_trajectories(ct.c_void_p(y.data_ptr()), y.shape[1], int(n_ant), y.shape[0], int(block_len),
                                      ct.c_void_p(ke.data_ptr()), ct.c_void_p(tb.data_ptr()), ke.numel(),
                                      ct.c_void_p(p.data_ptr()), _stream_handle(stream))
    if rc != OK:
        raise DdxError(rc, "ddx_chimg_trajectories")
    return p


def chimg_gradient_sums(y, n_ant, block_len, grads, lengths, stream=None):
    """Partial sums along common-gradient trajectories: P [grads, lengths, blocks]
    (complex64, device) over y [n_s, blocks]; lengths ascending."""
    import torch
    if y.dtype != torch.complex64 or y.dim() != 2:
        raise DdxError(EINVAL, "y must be complex64 [n_s, blocks]")
    ln = np.asarray(lengths, dtype=np.int32)
    if ln.size == 0 or np.any(ln < 1) or np.any(np.diff(ln) < 0):
        raise DdxError(EINVAL, "lengths must be ascending and >= 1")
    y = y.contiguous()
    gr = torch.as_tensor(np.asarray(grads, dtype=np.float64), device=y.device)
    lt = torch.as_tensor(ln, device=y.device)
    p = torch.empty((gr.numel(), lt.numel(), y.shape[1]), dtype=torch.complex64, device=y.device)
    rc = lib().ddx_chimg_gradient_sums(ct.c_void_p(y.data_ptr()), y.shape[1], int(n_ant), y.shape[0],
                                       int(block_len), ct.c_void_p(gr.data_ptr()), gr.numel(),
                                       ct.c_void_p(lt.data_ptr()), lt.numel(), ct.c_void_p(p.data_ptr()),
                                       _stream_handle(stream))
    if rc != OK:
        raise DdxError(rc, "ddx_chimg_gradient_sums")
    return p


def chimg_cells(positions, spacing, n_cells):
    """Cells of a line of antennas at ascending positions: (cell_ptr [n_cells + 1],
    cell_pairs [n_pairs, 2]) int32 host arrays (see ddx_chimg_cells)."""
    x = np.ascontiguousarray(positions, dtype=np.float64)
    ptr = np.zeros(int(n_cells) + 1, dtype=np.int32)
    prs = np.zeros((max(1, x.size * (x.size - 1) // 2), 2), dtype=np.int32)
    cnt = ct.c_int32()
    ip = ct.POINTER(ct.c_int32)
    rc = lib().ddx_chimg_cells(x.size, x.ctypes.data_as(ct.POINTER(ct.c_double)), float(spacing), int(n_cells),
                               ptr.ctypes.data_as(ip), prs.ctypes.data_as(ip), ct.byref(cnt))
    if rc != OK:
        raise DdxError(rc, "ddx_chimg_cells")
    return ptr, prs[:cnt.value]


def chimg_preintegrate_cells(volts, block_len, n_s, cell_ptr, cell_pairs, stream=None):
    """The Chimageator pre-integrator over gridding cells (ddx_chimg_preintegrate_cells):
    volts device complex64 [M, n]; returns device complex64 Y [n_s, n // block_len]."""
    import torch
    if volts.dtype != torch.complex64 or volts.dim() != 2:
        raise DdxError(EINVAL, "volts must be complex64 [M, n]")
    volts = volts.contiguous()
    M, n = volts.shape
    ptr = torch.as_tensor(np.ascontiguousarray(cell_ptr, dtype=np.int32), device=volts.device)
    prs = torch.as_tensor(np.ascontiguousarray(cell_pairs, dtype=np.int32).reshape(-1, 2), device=volts.device)
    if prs.numel() == 0:
        prs = torch.zeros((1, 2), dtype=torch.int32, device=volts.device)
    y = torch.empty((n_s, n // block_len), dtype=torch.complex64, device=volts.device)
    rc = lib().ddx_chimg_preintegrate_cells(ct.c_void_p(volts.data_ptr()), M, n, int(block_len), int(n_s),
                                            ptr.numel() - 1, ct.c_void_p(ptr.data_ptr()), ct.c_void_p(prs.data_ptr()),
                                            ct.c_void_p(y.data_ptr()), _stream_handle(stream))
    if rc != OK:
        raise DdxError(rc, "ddx_chimg_preintegrate_cells")
    return y


def chimg_sampling_blocks(k_end, t_blocks, kappa_t0):
    """Blocks per integrated sample of a trajectory (ddx_chimg_sampling_blocks)."""
    r = lib().ddx_chimg_sampling_blocks(float(k_end), int(t_blocks), float(kappa_t0))
    if r < 0:
        raise DdxError(r, "ddx_chimg_sampling_blocks")
    return r


def chimg_trajectories_ext(y, n_ant, block_len, k_end, t_blocks, a_blocks=None, half_width=0, stream=None):
    """Widened (2F + 1 bins, F = half_width) and sampled (a_blocks per integrated
    sample) trajectory sums P [trials, blocks] (complex64, device) over y [n_s, blocks]."""
    import torch
    if y.dtype != torch.complex64 or y.dim() != 2:
        raise DdxError(EINVAL, "y must be complex64 [n_s, blocks]")
    y = y.contiguous()
    ke = torch.as_tensor(np.asarray(k_end, dtype=np.float64), device=y.device)
    tb = torch.as_tensor(np.asarray(t_blocks, dtype=np.int32), device=y.device)
    ab = None if a_blocks is None else torch.as_tensor(np.asarray(a_blocks, dtype=np.int32), device=y.device)
    p = torch.empty((ke.numel(), y.shape[1]), dtype=torch.complex64, device=y.device)
    rc = lib().ddx_chimg_trajectories_ext(ct.c_void_p(y.data_ptr()), y.shape[1], int(n_ant), y.shape[0],
                                          int(block_len), ct.c_void_p(ke.data_ptr()), ct.c_void_p(tb.data_ptr()),
                                          None if ab is None else ct.c_void_p(ab.data_ptr()), int(half_width),
                                          ke.numel(), ct.c_void_p(p.data_ptr()), _stream_handle(stream))
    if rc != OK:
        raise DdxError(rc, "ddx_chimg_trajectories_ext")
    return p


def chimg_cells_2d(positions, spacing, max_cells=1024):
    """Planar gridding tables (ddx_chimg_cells_2d): (cell_ptr, cell_pairs [pairs, 2],
    cell_uv [cells, 2]) as int32 numpy arrays."""
    pos = np.ascontiguousarray(positions, dtype=np.float64)
    m = pos.shape[0]
    ptr = np.zeros(max_cells + 1, dtype=np.int32)
    pairs = np.zeros(max(m * (m - 1), 2), dtype=np.int32)
    uv = np.zeros(2 * max_cells, dtype=np.int32)
    nc, npairs = ct.c_int32(0), ct.c_int32(0)
    rc = lib().ddx_chimg_cells_2d(m, pos.ctypes.data_as(ct.POINTER(ct.c_double)), float(spacing), int(max_cells),
                                  ct.byref(nc), ptr.ctypes.data_as(ct.POINTER(ct.c_int32)),
                                  pairs.ctypes.data_as(ct.POINTER(ct.c_int32)),
                                  uv.ctypes.data_as(ct.POINTER(ct.c_int32)), ct.byref(npairs))
    if rc != OK:
        raise DdxError(rc, "ddx_chimg_cells_2d")
    return ptr[:nc.value + 1].copy(), pairs[:2 * npairs.value].reshape(-1, 2).copy(), uv[:2 * nc.value].reshape(-1,
                                                                                                             2).copy()


def chimg_preintegrate_2d(volts, block_len, n_s, cells, stream=None):
    """Planar pre-integrator: volts device complex64 [M, n], cells from chimg_cells_2d;
    returns device complex64 Y [n_s * n_s, n // block_len] (bin ku n_s + kv)."""
    import torch
    if volts.dtype != torch.complex64 or volts.dim() != 2:
        raise DdxError(EINVAL, "volts must be complex64 [M, n]")
    volts = volts.contiguous()
    M, n = volts.shape
    ptr, pairs, uv = (torch.as_tensor(np.ascontiguousarray(a), device=volts.device) for a in cells)
    y = torch.empty((n_s * n_s, n // block_len), dtype=torch.complex64, device=volts.device)
    rc = lib().ddx_chimg_preintegrate_2d(ct.c_void_p(volts.data_ptr()), M, n, int(block_len), int(n_s),
                                         uv.shape[0], ct.c_void_p(ptr.data_ptr()), ct.c_void_p(pairs.data_ptr()),
                                         ct.c_void_p(uv.data_ptr()), ct.c_void_p(y.data_ptr()), _stream_handle(stream))
    if rc != OK:
        raise DdxError(rc, "ddx_chimg_preintegrate_2d")
    return y


def chimg_trajectories_2d(y, n_s, block_len, cell_uv, k_end, t_blocks, stream=None):
    """Planar trajectory sums P [trials, blocks] (complex64, device) over the planar
    pre-integrator's y; k_end [trials, 2] end bins (ku, kv)."""
    import torch
    if y.dtype != torch.complex64 or y.dim() != 2 or y.shape[0] != n_s * n_s:
        raise DdxError(EINVAL, "y must be complex64 [n_s * n_s, blocks]")
    y = y.contiguous()
    ke = torch.as_tensor(np.ascontiguousarray(k_end, dtype=np.float64).reshape(-1, 2), device=y.device)
    tbn = np.asarray(t_blocks, dtype=np.int32)
    tb = torch.as_tensor(tbn, device=y.device)
    uv = torch.as_tensor(np.ascontiguousarray(cell_uv, dtype=np.int32), device=y.device)
    max_t = int(tbn.max())
    bins = torch.empty((tbn.size, max_t), dtype=torch.int32, device=y.device)
    w = torch.empty((tbn.size, max_t), dtype=torch.complex64, device=y.device)
    p = torch.empty((tbn.size, y.shape[1]), dtype=torch.complex64, device=y.device)
    rc = lib().ddx_chimg_trajectories_2d(ct.c_void_p(y.data_ptr()), y.shape[1], int(n_s), int(block_len),
                                         uv.shape[0], ct.c_void_p(uv.data_ptr()), ct.c_void_p(ke.data_ptr()),
                                         ct.c_void_p(tb.data_ptr()), tbn.size, max_t, ct.c_void_p(bins.data_ptr()),
                                         ct.c_void_p(w.data_ptr()), ct.c_void_p(p.data_ptr()), _stream_handle(stream))
    if rc != OK:
        raise DdxError(rc, "ddx_chimg_trajectories_2d")
    return p
