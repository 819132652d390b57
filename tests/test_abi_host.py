"""Host-side checks of the C ABI: symbols, argument validation, call order.

None of these calls touches the GPU: plan creation validates and allocates
nothing on the device, and every failure below is detected on the host first.
"""
import ctypes as ct
import os
import re

import numpy as np
import pytest

import paper_1109_3186_amd as ddx
from paper_1109_3186_amd import binding

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "ddx.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ddx_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 9
    lib = ct.CDLL(ddx.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(binding.SIGNATURES)


def _desc(**kw):
    fc = np.array(kw.pop("fc", [1.4e9, 1.401e9]), dtype=np.float64)
    d = binding.Desc()
    d.n_ant = kw.pop("n_ant", 4)
    d.n_chan = kw.pop("n_chan", len(fc))
    d.chan_freq_hz = fc.ctypes.data_as(ct.POINTER(ct.c_double))
    d.samp_rate_hz = kw.pop("fs", 1e6)
    d.sideband = kw.pop("sideband", 1)
    d.in_dtype = kw.pop("in_dtype", 0)
    d.corr_dtype = kw.pop("corr_dtype", 0)
    d.dump_len = kw.pop("dump_len", 64)
    d.k_dm = kw.pop("k_dm", 0.0)
    d.max_block_samples = kw.pop("max_block", 1 << 16)
    d.max_device_bytes = kw.pop("max_bytes", 0)
    d.out_mode = kw.pop("out_mode", 0)
    assert not kw
    return d, fc


def _create(**kw):
    d, fc = _desc(**kw)
    h = ct.c_void_p()
    rc = ddx.lib().ddx_plan_create(ct.byref(d), ct.byref(h))
    return rc, h


@pytest.mark.parametrize("bad", [
    {"n_ant": 0}, {"n_chan": 0}, {"fs": 0.0}, {"fs": float("nan")}, {"sideband": 0}, {"in_dtype": 5},
    {"corr_dtype": 9}, {"dump_len": 0}, {"max_block": 0}, {"out_mode": 3}, {"k_dm": -1.0},
    {"fc": [1.4e9, float("inf")]}, {"fc": [1.4e9, 1e5]},
])
def test_create_rejects_invalid_fields(bad):
    rc, h = _create(**bad)
    assert rc == ddx.EINVAL and not h.value


def test_create_null_arguments():
    d, _ = _desc()
    assert ddx.lib().ddx_plan_create(None, None) == ddx.EINVAL
    assert ddx.lib().ddx_plan_create(ct.byref(d), None) == ddx.EINVAL


def test_call_order_and_argument_errors():
    rc, h = _create()
    assert rc == ddx.OK and h.value
    L = ddx.lib()
    lay = binding.Layout()
    assert L.ddx_get_layout(h, ct.byref(lay)) == ddx.ESTATE
    assert L.ddx_process_block(h, None, 0, 0, None) == ddx.ESTATE
    first, nd = ct.c_int64(), ct.c_int64()
    assert L.ddx_fetch_visibilities(h, None, 0, ct.byref(first), ct.byref(nd), None) == ddx.ESTATE
    assert L.ddx_set_active_dms(h, -1, None) == ddx.ESTATE
    dm = np.array([0.0, -1.0])
    assert L.ddx_set_dm_trials(h, -1, dm.ctypes.data_as(ct.POINTER(ct.c_double)), 2) == ddx.EINVAL
    assert b"DM[1]" in L.ddx_last_error(h)
    dm = np.array([0.0, float("nan")])
    assert L.ddx_set_dm_trials(h, -1, dm.ctypes.data_as(ct.POINTER(ct.c_double)), 2) == ddx.EINVAL
    assert L.ddx_set_dm_trials(h, -1, None, 1) == ddx.EINVAL
    assert L.ddx_set_dm_trials(h, 7, dm.ctypes.data_as(ct.POINTER(ct.c_double)), 1) == ddx.EINVAL
    # a DM so large the smear needs more than the supported FFT length
    dm = np.array([1e6])
    assert L.ddx_set_dm_trials(h, -1, dm.ctypes.data_as(ct.POINTER(ct.c_double)), 1) == ddx.EUNSUPPORTED
    # setting only one channel leaves the plan not ready (no device work yet)
    dm = np.array([10.0])
    assert L.ddx_set_dm_trials(h, 0, dm.ctypes.data_as(ct.POINTER(ct.c_double)), 1) == ddx.OK
    assert L.ddx_get_layout(h, ct.byref(lay)) == ddx.ESTATE
    assert L.ddx_plan_destroy(h) == ddx.OK


def test_fft_too_short_for_smear():
    fc = np.array([0.7e9])
    d, _ = _desc(fc=fc, n_chan=1)
    fl = np.array([1024], dtype=np.int32)
    d.fft_len = fl.ctypes.data_as(ct.POINTER(ct.c_int32))
    h = ct.c_void_p()
    assert ddx.lib().ddx_plan_create(ct.byref(d), ct.byref(h)) == ddx.OK
    dm = np.array([500.0])
    assert ddx.lib().ddx_set_dm_trials(h, -1, dm.ctypes.data_as(ct.POINTER(ct.c_double)), 1) == ddx.EINVAL
    ddx.lib().ddx_plan_destroy(h)


def test_unsupported_and_bad_fft_lengths():
    d, fc = _desc()
    fl = np.array([3000, 0], dtype=np.int32)
    d.fft_len = fl.ctypes.data_as(ct.POINTER(ct.c_int32))
    h = ct.c_void_p()
    assert ddx.lib().ddx_plan_create(ct.byref(d), ct.byref(h)) == ddx.EINVAL
    rc, h = _create(n_ant=2000)
    assert rc == ddx.EUNSUPPORTED


def test_strerror_and_null_plan():
    L = ddx.lib()
    for s in (ddx.OK, ddx.EINVAL, ddx.ENOMEM, ddx.EDEVICE, ddx.ESTATE, ddx.ESIZE, ddx.EFULL, ddx.EUNSUPPORTED):
        assert L.ddx_strerror(s) and L.ddx_strerror(s) != b"unknown status"
    assert L.ddx_plan_destroy(None) == ddx.OK
    assert L.ddx_process_block(None, None, 0, 0, None) == ddx.EINVAL
    assert L.ddx_set_dm_trials(None, 0, None, 0) == ddx.EINVAL


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of ddx_desc, ddx_layout and ddx_profile have the C sizes and field offsets."""
    structs = {"ddx_desc": binding.Desc, "ddx_layout": binding.Layout, "ddx_profile": binding.Profile}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ddx.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            if f == "pad":
                continue
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines.append("return 0; }")
    src = tmp_path / "sizes.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "sizes"
    import subprocess
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(ln.split()[:2]): int(ln.split()[2]) for ln in out if ln}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ct.sizeof(py), cname
        for f, _ in py._fields_:
            if f != "pad":
                assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_autotune_dm_sampling_keeps_the_largest():
    from paper_1109_3186_amd.autotune import _sample_dms
    d = np.linspace(0, 3000, 1536, endpoint=False)[::-1].copy()  # largest first
    s = _sample_dms(d, 16)
    assert d.max() in s and len(s) <= 17 and len(np.unique(s)) == len(s)
    assert np.array_equal(_sample_dms(d[:5], 16), d[:5])


def test_chirp_create_rejects_invalid_arguments():
    """Argument checks of ddx_chirp_create run before any device call."""
    L = ct.CDLL(ddx.LIB_PATH)
    for args in [(1, 64, 16, 4, 1000), (2000, 64, 16, 4, 1000), (4, 60, 16, 4, 1000), (4, 64, 0, 4, 1000),
                 (4, 64, 16, -1, 1000), (4, 64, 16, 32, 1000), (4, 64, 16, 4, 63)]:
        h = ct.c_void_p()
        assert L.ddx_chirp_create(*[ct.c_int32(a) for a in args[:4]], ct.c_int64(args[4]), ct.byref(h)) == \
            binding.EINVAL, args
        assert not h.value
    assert L.ddx_chirp_create(4, 64, 16, 4, ct.c_int64(1000), None) == binding.EINVAL
    assert L.ddx_chirp_destroy(None) == binding.OK
    assert L.ddx_chirp_preintegrate(None, None, ct.c_int64(0), None, None) == binding.EINVAL


def test_chirp_bank_create_rejects_invalid_arguments():
    L = ct.CDLL(ddx.LIB_PATH)
    for args in [(1, 64, 4, 16, 4, 1000), (4, 60, 4, 16, 4, 1000), (4, 64, 0, 16, 4, 1000), (4, 64, 65, 16, 4, 10 ** 6),
                 (4, 64, 4, 16, 40, 1000), (4, 64, 4, 16, 4, 255)]:
        h = ct.c_void_p()
        rc = L.ddx_chirp_bank_create(*[ct.c_int32(a) for a in args[:5]], ct.c_int64(args[5]), ct.byref(h))
        assert rc == binding.EINVAL, args
        assert not h.value
    assert L.ddx_chirp_bank_destroy(None) == binding.OK
    assert L.ddx_chirp_bank_run(None, None, ct.c_int64(0), None, None) == binding.EINVAL
    assert L.ddx_chirp_bank_set_pair_bins(None, None) == binding.EINVAL
    assert L.ddx_chirp_set_pair_bins(None, None) == binding.EINVAL


def test_image_create_rejects_invalid_arguments():
    L = ct.CDLL(ddx.LIB_PATH)
    dp = ct.POINTER(ct.c_double)
    ant = np.zeros((4, 3))
    ant[:, 0] = np.arange(4) * 100.0
    pix = np.array([[0.01, 0.02], [0.0, 0.0]])
    good = dict(n_ant=4, n_pix=2, fdot=1e10, fs=1e6, N=256, L=16, kmax=10, F=2)

    def create(ant=ant, pix=pix, **kw):
        a = dict(good, **kw)
        h = ct.c_void_p()
        ant = np.ascontiguousarray(ant, dtype=np.float64)
        pix = np.ascontiguousarray(pix, dtype=np.float64)
        rc = L.ddx_image_create(ct.c_int32(a["n_ant"]), ant.ctypes.data_as(dp), ct.c_int32(a["n_pix"]),
                                pix.ctypes.data_as(dp), ct.c_double(a["fdot"]), ct.c_double(a["fs"]),
                                ct.c_int32(a["N"]), ct.c_int32(a["L"]), ct.c_int32(a["kmax"]), ct.c_int32(a["F"]),
                                ct.byref(h))
        assert not h.value
        return rc

    for kw in [dict(n_ant=1), dict(n_pix=0), dict(N=250), dict(L=0), dict(kmax=-1), dict(kmax=641, N=4096),
               dict(kmax=200), dict(F=9), dict(F=-1), dict(fs=0.0), dict(fdot=float("inf")), dict(N=2 ** 20, L=8)]:
        assert create(**kw) == binding.EINVAL, kw
    assert create(pix=np.array([[0.8, 0.7], [0.0, 0.0]])) == binding.EINVAL   # l^2 + m^2 >= 1
    assert create(pix=np.array([[np.nan, 0.0], [0.0, 0.0]])) == binding.EINVAL
    bad = ant.copy()
    bad[2, 1] = np.inf
    assert create(ant=bad) == binding.EINVAL
    assert L.ddx_image_destroy(None) == binding.OK
    assert L.ddx_image_run(None, None, ct.c_int64(0), ct.c_int64(0), ct.c_int32(1), None, None, None) == binding.EINVAL
    n = ct.c_int64()
    assert L.ddx_image_output_count(None, ct.c_int64(5), ct.c_int32(2), ct.byref(n)) == binding.EINVAL


def test_incoherent_delays_match_the_oracle_and_validate():
    """The host delay table (Eq. dmdelay, FP64, ties to even) equals the oracle's
    bit for bit; invalid arguments are rejected before any device work."""
    from oracle import incoherent as oinc
    f = 1.2005e9 + 1e6 * np.arange(64)[::-1]
    dms = np.arange(256) * 2000.0 / 256
    got = binding.incoherent_delays(f, 1e-3, dms)
    assert np.array_equal(got, oinc.dm_delays(f, 1e-3, dms))
    with pytest.raises(binding.DdxError):
        binding.incoherent_delays(f, 0.0, dms)
    with pytest.raises(binding.DdxError):
        binding.incoherent_delays(f, 1e-3, [-1.0])
    L = ct.CDLL(ddx.LIB_PATH)
    assert L.ddx_tree_dedisperse(None, ct.c_int32(64), ct.c_int64(10), None, None, None) == binding.EINVAL
    dummy = ct.c_void_p(8)   # never dereferenced: the size check fails first
    assert L.ddx_tree_dedisperse(dummy, ct.c_int32(48), ct.c_int64(10), dummy, dummy, None) == binding.EINVAL
    assert L.ddx_tree_dedisperse(dummy, ct.c_int32(64), ct.c_int64(10), dummy, None, None) == binding.EINVAL
    assert L.ddx_incoherent_dedisperse(None, ct.c_int32(4), ct.c_int64(10), None, ct.c_int32(2), None,
                                       ct.c_int64(5), None) == binding.EINVAL
    assert L.ddx_power_beam(None, ct.c_int32(4), ct.c_int32(2), ct.c_int64(10), ct.c_int32(2), None,
                            None) == binding.EINVAL


def test_chimageator_entry_points_validate():
    L = ct.CDLL(ddx.LIB_PATH)
    d = ct.c_void_p(8)   # never dereferenced: the argument checks fail first
    assert L.ddx_chimg_preintegrate(d, ct.c_int32(1), ct.c_int64(100), ct.c_int32(4), ct.c_int32(16), ct.c_int32(1),
                                    d, None) == binding.EINVAL            # one antenna
    assert L.ddx_chimg_preintegrate(d, ct.c_int32(258), ct.c_int64(100), ct.c_int32(4), ct.c_int32(16),
                                    ct.c_int32(1), d, None) == binding.EINVAL   # above 257
    assert L.ddx_chimg_preintegrate(d, ct.c_int32(8), ct.c_int64(100), ct.c_int32(4), ct.c_int32(24), ct.c_int32(1),
                                    d, None) == binding.EINVAL            # N_s not a power of two
    assert L.ddx_chimg_preintegrate(d, ct.c_int32(8), ct.c_int64(100), ct.c_int32(4), ct.c_int32(2048),
                                    ct.c_int32(1), d, None) == binding.EINVAL   # N_s above 1024
    assert L.ddx_chimg_trajectories(None, ct.c_int64(10), ct.c_int32(8), ct.c_int32(16), ct.c_int32(4), d, d,
                                    ct.c_int32(1), d, None) == binding.EINVAL
    assert L.ddx_chimg_gradient_sums(d, ct.c_int64(10), ct.c_int32(8), ct.c_int32(16), ct.c_int32(4), d,
                                     ct.c_int32(0), d, ct.c_int32(1), d, None) == binding.EINVAL
    with pytest.raises(binding.DdxError):
        binding.chimg_gradient_sums(_FakeTensor(), 8, 4, [0.1], [5, 3])


class _FakeTensor:
    """Stands in for a device tensor in a check that fails before any device work."""
    import torch as _t
    dtype = _t.complex64

    def dim(self):
        return 2


def test_chimageator_cells_match_the_oracle():
    """The host cell table equals the oracle's gridding of the same positions."""
    from oracle import chimageator as ocg
    rng = np.random.Generator(np.random.PCG64(77))
    x = np.sort(rng.uniform(0, 600.0, 12))
    x = x[np.concatenate([[True], np.diff(x) > 0])]
    ptr, prs = binding.chimg_cells(x, 25.0, 20)
    ref = ocg.nearest_cells(x, 25.0)
    for l in range(1, 21):
        got = [tuple(p) for p in prs[ptr[l - 1]:ptr[l]]]
        assert got == ref.get(l, []), l
    with pytest.raises(binding.DdxError):
        binding.chimg_cells([0.0, 5.0, 3.0], 1.0, 4)      # not ascending


def test_planar_cells_and_sampling_rule_on_the_host():
    """ddx_chimg_cells_2d and ddx_chimg_sampling_blocks are host code: against the
    oracle's nearest cells (half plane, turned pairs, cell order) and its sampling rule."""
    from oracle import chimageator as ocg
    rng = np.random.Generator(np.random.PCG64(870))
    for m, jitter in [(7, 0.0), (30, 9.0)]:
        pos = rng.integers(0, 9, (m, 2)) * 30.0 + rng.uniform(-jitter, jitter, (m, 2))
        ptr, pairs, uv = ddx.chimg_cells_2d(pos, 30.0)
        got = {(int(uv[c, 0]), int(uv[c, 1])): [tuple(int(v) for v in pairs[b]) for b in range(ptr[c], ptr[c + 1])]
               for c in range(uv.shape[0])}
        ref = ocg.nearest_cells_2d(pos, 30.0)
        assert got == ref and [tuple(r) for r in uv] == sorted(ref)
    with pytest.raises(ddx.DdxError):
        ddx.chimg_cells_2d(rng.uniform(0, 1000, (20, 2)), 1.0, max_cells=10)
    for args in [(9.0, 240, 5.0), (0.0, 240, 5.0), (100.0, 240, 5.0), (-3.3, 77, 2.5)]:
        assert ddx.chimg_sampling_blocks(*args) == ocg.sampling_blocks(*args)


def _smear_half(fc, fs, dm):
    import math

    import oracle
    early, late = oracle.smear_samples(fc, fs, dm)
    return int(math.ceil(max(early, late)))


@pytest.mark.parametrize("fc,dmax,nd,L", [(1.2e9, 2000.0, 256, 1000), (0.7e9, 3000.0, 1536, 1000),
                                          (1.4e9, 100.0, 16, 64), (0.732e9, 3000.0, 100, 1000)])
def test_blocking_classes_on_the_host(fc, dmax, nd, L):
    """The blocking rule without a device (ddx_plan_blocking).  "single": every DM gets
    the oracle's rule at the channel's largest DM.  "auto": the DMs, sorted, fall into
    contiguous classes whose blocking is the oracle's rule at the class's largest DM
    and the class's own length, so every DM's overlap covers its own smear on both
    sides; cuts lie at multiples of 16 sorted DMs; a requested FFT length keeps one
    class."""
    import oracle
    from paper_1109_3186_amd import plan_blocking
    rng = np.random.default_rng(int(fc) % 1000 + nd)
    dms = rng.permutation(np.linspace(0.0, dmax, nd))  # any order
    n, v, l, k = plan_blocking([fc], 1e6, L, dms, dm_classes="single")
    ref = oracle.blocking(fc, 1e6, dms.max(), L)
    assert k == 1 and set(n) == {ref["fft_len"]} and set(v) == {ref["valid"]} and set(l) == {ref["lead"]}
    n, v, l, k = plan_blocking([fc], 1e6, L, dms)
    order = np.argsort(dms, kind="stable")
    keys = [(n[d], v[d], l[d]) for d in order]
    cuts = [i for i in range(1, nd) if keys[i] != keys[i - 1]]
    assert len(cuts) == k - 1 and all(c % 16 == 0 for c in cuts)
    for lo, hi in zip([0] + cuts, cuts + [nd]):
        cls = order[lo:hi]
        r = oracle.blocking(fc, 1e6, dms[cls].max(), L, fft_len=int(n[cls[0]]))
        assert keys[lo] == (r["fft_len"], r["valid"], r["lead"])
    for d in range(nd):
        a = _smear_half(fc, 1e6, dms[d])
        assert v[d] % L == 0 and v[d] >= L and 256 <= n[d] <= 1 << 18 and n[d] & (n[d] - 1) == 0
        assert l[d] >= a and n[d] - v[d] - l[d] >= a
    n2, _, _, k2 = plan_blocking([fc], 1e6, L, dms, fft_len=1 << 15 if dmax < 2500 else 1 << 18)
    assert k2 == 1 and len(set(n2)) == 1


def test_blocking_classes_reject_like_the_plan():
    from paper_1109_3186_amd import DdxError, plan_blocking
    with pytest.raises(DdxError):  # smear beyond 2^18
        plan_blocking([0.3e9], 1e6, 1000, [0.0, 5000.0])
    with pytest.raises(DdxError):  # negative DM
        plan_blocking([1.2e9], 1e6, 1000, [-1.0])
    with pytest.raises(DdxError):  # channel out of range
        plan_blocking([1.2e9], 1e6, 1000, [1.0], chan=1)


def test_blocking_cost_table_steers_the_classes():
    """A cost table in the descriptor replaces the built-in one: made cheap only at
    2^15, every class takes 32768 points; a non-positive entry is rejected."""
    from paper_1109_3186_amd import DdxError, plan_blocking
    dms = np.linspace(0.0, 2000.0, 256)
    cost = np.full((2, 11), 50.0)
    cost[:, 7] = 1.0
    n, v, l, k = plan_blocking([1.2e9], 1e6, 1000, dms, cost_ps=cost)
    assert set(n.tolist()) == {1 << 15}
    auto_n, _, _, _ = plan_blocking([1.2e9], 1e6, 1000, dms)
    assert len(set(auto_n.tolist())) > 1
    bad = cost.copy()
    bad[1, 3] = 0.0
    with pytest.raises(DdxError):
        plan_blocking([1.2e9], 1e6, 1000, dms, cost_ps=bad)


def test_cnn_create_rejects_bad_shapes():
    """ddx_cnn_create validates before touching the device: bins not a multiple of 64,
    no rows, and more rows than the convolutions' grids take are refused."""
    import ctypes as ct

    from paper_1109_3186_amd.binding import lib
    h = ct.c_void_p()
    for n_dm, n_bins, tiles in ((256, 100, 1), (0, 1024, 1), (256, 1024, 0), (4096, 1024, 16), (65536, 64, 1)):
        assert lib().ddx_cnn_create(n_dm, n_bins, tiles, ct.byref(h)) == -1, (n_dm, n_bins, tiles)
    assert lib().ddx_cnn_set_precision(None, 1) == -1
    assert lib().ddx_cnn_get_activations(None, 1, None, 0) == -1


def test_wave_size_above_the_grid_limit_is_refused():
    """A wave holds at most 65535 units (one chirp grid row per (channel, DM) of a
    wave): larger requests fail at plan creation, before any device call."""
    import pytest as _pytest

    from paper_1109_3186_amd import DdxError, Plan
    with _pytest.raises(DdxError) as e:
        Plan(4, [1.2e9], 1e6, 1000, max_block_samples=1 << 16, wave_units=65536)
    assert e.value.status == -1
    Plan(4, [1.2e9], 1e6, 1000, max_block_samples=1 << 16, wave_units=65535).close()
