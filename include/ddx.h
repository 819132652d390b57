/* ddx: coherent-dedispersion correlator for AMD MI355X (gfx950).
 *
 * The pre-integrator stage of an antenna-coherent search for dispersed radio
 * pulses (Bannister & Cornwell 2011, "The Chirpolator and The Chimageator"):
 *
 *   1. each antenna's complex baseband voltages (Sec. 3.2: complex Nyquist
 *      sampling, f_s = channel bandwidth) are coherently dedispersed for every
 *      trial DM: convolved with the inverse of the interstellar medium's
 *      response (Sec. 2.3.2), derived from the delay law of Eq. dmdelay
 *      (Sec. 2.1), using overlap-save FFT blocks;
 *   2. every antenna pair is multiplied, one voltage by the other's conjugate
 *      (the "mixing" of Sec. 3.2, Eq. xpq), and integrated and dumped at a
 *      fixed cadence (the integrate-and-dump boundary of Sec. 5.1), giving
 *      per-DM visibilities.  At DM = 0 a dump equals the k = 0 term of the block
 *      partial DFT of Appendix A.3 (Eq. block_cic).
 *
 * Conventions shared by all calls:
 *   - every function returns DDX_OK (0) or a negative DDX_E* status and never
 *     aborts; ddx_last_error() holds a message for the last failure of a plan;
 *   - units: Hz, seconds, pc cm^-3 as double; sample counts as int64_t;
 *   - a plan is not thread-safe; separate plans are independent;
 *   - memory owned by the plan: spectra, chirp tables, dedispersed voltages,
 *     the dump ring, the input history.  Memory owned by the caller: inputs,
 *     outputs, streams (a hipStream_t passed as void*, NULL = default stream).
 *
 * Readings where the paper is silent (the filter's form and sign, bin
 * frequencies, blocking, normalisation, baseline order) are stated at the
 * calls that depend on them.
 */
#ifndef DDX_H
#define DDX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define DDX_OK 0
#define DDX_EINVAL (-1)       /* invalid argument */
#define DDX_ENOMEM (-2)       /* device allocation failed or max_device_bytes exceeded */
#define DDX_EDEVICE (-3)      /* a HIP call or kernel launch failed */
#define DDX_ESTATE (-4)       /* call not allowed in the plan's current state */
#define DDX_ESIZE (-5)        /* caller buffer too small */
#define DDX_EFULL (-6)        /* unfetched dumps would be overwritten */
#define DDX_EUNSUPPORTED (-7) /* valid request this library does not implement */

/* Input sample formats: interleaved (re, im). */
#define DDX_IN_CI8 0  /* int8 re, int8 im: 2 bytes per sample */
#define DDX_IN_CF32 1 /* float re, float im: 8 bytes per sample */

/* Correlator input formats (the dedispersed voltages). */
#define DDX_CORR_F32 0  /* FP32 voltages; products from a two-term binary16 split (hi*hi + hi*lo
                           + lo*hi) on FP16 MFMA, FP32 accumulate: normalised visibility error
                           ~1e-6 (a plain FP32 sum would give ~1e-7).  The split's range follows
                           each (channel, DM, block): a block whose largest component of s y
                           exceeds 2^15 is split at a smaller power of two, so later level
                           changes cannot overflow binary16 */
#define DDX_CORR_F16 1  /* voltages x scale rounded to IEEE binary16 (RNE, saturating) */
#define DDX_CORR_E4M3 2 /* voltages x scale rounded to OCP FP8 E4M3 (RNE, saturating to +-448) */

/* Visibility layout within one dump record. */
#define DDX_OUT_PACKED 0 /* upper triangle incl. autos, b(i,j) = i M - i(i-1)/2 + (j - i) */
#define DDX_OUT_FULL 1   /* full M x M, row-major, V_ji = conj(V_ij) */

/* ddx_process_block flags. */
#define DDX_FLUSH 1 /* end of stream: zero-pad after the last sample and finish */

typedef struct ddx_desc {
  int32_t n_ant;               /* M antennas, 1 <= M <= 1024 (more: DDX_EUNSUPPORTED) */
  int32_t n_chan;              /* C >= 1 channels */
  const double* chan_freq_hz;  /* [C] sky frequency of each channel's DC bin, > samp_rate/2 */
  double samp_rate_hz;         /* complex sample rate = channel bandwidth, > 0 */
  int32_t sideband;            /* +1: bin offset f is sky f_c + f; -1: sky f_c - f */
  int32_t in_dtype;            /* DDX_IN_* */
  int32_t corr_dtype;          /* DDX_CORR_* */
  int32_t dump_len;            /* L >= 1 samples per dump */
  const int32_t* fft_len;      /* [C] power-of-two FFT lengths, or NULL / 0 entries = auto */
  double k_dm;                 /* dispersion constant in s Hz^2 cm^3/pc; 0 = 4.148808e15 */
  int64_t max_block_samples;   /* largest n one ddx_process_block call accepts, >= 1 */
  size_t max_device_bytes;     /* cap on plan-owned device memory, 0 = none */
  int32_t out_mode;            /* DDX_OUT_* */
  const float* chan_scale;     /* [C] power-of-two correlator-input scales, or NULL = rule below */
  /* Schedule (all 0 = automatic; see ddx_process_block for the work list): */
  int32_t wave_units;          /* (channel, DM, block) units per wave, 0 (automatic) .. 65535 */
  int32_t dm_group;            /* DMs of one channel run back to back on each block, >= 0 */
  /* Dump records (see ddx_fetch_visibilities): */
  int32_t compact_records;     /* 0: every (channel, DM) in every record; 1: only the active ones */
  int32_t max_record_pairs;    /* compact records: capacity in (channel, DM) pairs, 0 = all */
  int64_t ring_dumps;          /* device dump ring capacity in dumps, 0 = enough for any call */
  /* Blocking (see ddx_set_dm_trials): */
  int32_t dm_classes;          /* 0: each channel's DMs in classes by the cost model; 1: one class per channel */
  int32_t pad;
  int64_t spectrum_bytes;      /* cap on the spectrum buffer, 0 = 32 GiB: a call runs its classes in
                                  batches whose spectra fit it (a class larger than it runs alone) */
  const double* cost_ps;       /* [2][11] cost model of the classes: picoseconds per transform point
                                  of the inverse (row 0) and forward (row 1) transforms for N = 2^8
                                  .. 2^18, each > 0 (measured by the autotuner); NULL = the built-in
                                  table (gfx950) */
} ddx_desc;

/* Scale rule when chan_scale is NULL (all correlator formats; the scale keeps
 * the binary16 halves of F32 and the F16/E4M3 values in range): s_c = 2^rint(log2(t / sigma_c)),
 * sigma_c the per-component RMS of channel c's samples [0, N_c - lead_c) over all
 * antennas (the in-stream part of its first block window), t = 32 for E4M3 (about
 * 10 sigma, and the int8 extreme 127 at sigma 16, stay below 448, the largest
 * finite E4M3 value) and t = 4 for F16 and F32.  It is
 * computed on the device when the channel's first block runs (so it does not
 * depend on how the stream is split) and exported by ddx_get_layout. */

typedef struct ddx_plan ddx_plan;

typedef struct ddx_layout {
  int32_t n_ant, n_chan, n_baselines, dump_len, out_mode, corr_dtype, in_dtype, sideband;
  double samp_rate_hz, k_dm;
  const double* chan_freq_hz;  /* [C] */
  const int32_t* fft_len;      /* [C] N_c of the class holding the channel's largest DM */
  const int32_t* valid;        /* [C] V_c of that class: outputs kept per block, a multiple of L */
  const int32_t* lead;         /* [C] lead_c of that class (the scale rule's window is [0, N_c - lead_c)) */
  const int32_t* n_dm;         /* [C] D_c trial DMs */
  const int64_t* dm_offset;    /* [C+1] prefix sums of D_c: index of (c, d) in the per-DM tables */
  const double* dm;            /* [dm_offset[C]] trial DMs, channel-major */
  const double* delay_s;       /* [dm_offset[C]] K DM / f_c^2: channel-centre delay behind infinite frequency */
  const int64_t* shift;        /* [dm_offset[C]] rint(K DM (f_c^-2 - f_top^-2) f_s): samples behind the highest channel */
  const float* scale;          /* [C] correlator-input scale s_c */
  const int32_t* record_pos;   /* [dm_offset[C]] slot of (c, d) in a dump record, -1 if not stored */
  int64_t record_pairs;        /* (channel, DM) slots per dump record */
  int64_t record_elems;        /* complex64 values per dump record = record_pairs * n_baselines */
  int64_t samples_in;          /* samples accepted so far per (channel, antenna) */
  int64_t dumps_ready;         /* dumps complete in every channel */
  int64_t dumps_fetched;       /* dumps already returned by ddx_fetch_visibilities */
  int64_t ring_dumps;          /* capacity of the device dump ring */
  size_t device_bytes;         /* plan-owned device memory */
  int32_t wave_units;          /* units per wave in use */
  int32_t dm_group;            /* DMs per block group in use */
  int32_t compact_records;     /* as in the descriptor */
  int32_t pad;
  /* Dump times (Sec. 5.1's integrate-and-dump cadence): dump m of channel c stands at
   * dump_t0_s + m dump_period_s seconds after the stream's first sample at the
   * channel centre, and at that minus delay_s[(c, d)] referred to infinite frequency
   * (see ddx_dump_times). */
  double dump_t0_s;            /* (L - 1) / (2 f_s): the mean time of dump 0's samples */
  double dump_period_s;        /* L / f_s */
  /* Blocking of every (channel, DM): that of its class (see ddx_set_dm_trials). */
  const int32_t* dm_fft_len;   /* [dm_offset[C]] N */
  const int32_t* dm_valid;     /* [dm_offset[C]] V, a multiple of L */
  const int32_t* dm_lead;      /* [dm_offset[C]] lead: block b reads samples [b V - lead, b V - lead + N) */
  int32_t n_classes;           /* blocking classes over all channels */
  int32_t pad2;
} ddx_layout;

/* Create a plan from a descriptor (copied; the caller's arrays may be freed).
 * Validates all fields and allocates nothing on the device.  *out is set only
 * on success.  Errors: EINVAL (bad field), ENOMEM (host allocation). */
int ddx_plan_create(const ddx_desc* desc, ddx_plan** out);

/* Set the trial DMs of one channel (chan >= 0) or of all (chan = -1): n_dm >= 1
 * finite values >= 0 in any order and spacing (uniform, or the geometric banks
 * of Appendix A.4, Eq. Ti).  When every channel has its list, fixes the
 * overlap-save blocking (the paper fixes none; Sec. 2.3.2 only asks for the
 * convolution with the inverse of the medium's response):
 *   - the half overlap a DM needs, A(DM) = ceil(max intra-channel smear) in
 *     samples, where the top edge f_c + f_s/2 arrives K DM (f_c^-2 - (f_c +
 *     f_s/2)^-2) before the centre and the bottom edge K DM ((f_c - f_s/2)^-2 -
 *     f_c^-2) after it (Eq. dmdelay);
 *   - a class of DMs shares one blocking, that of its largest DM: FFT length N,
 *     V = L floor((N - 2 A) / L) outputs kept per block, lead = floor((N - V)/2);
 *   - with the descriptor's FFT length for the channel, or dm_classes = 1, all
 *     of the channel's DMs form one class, with that length or else the smallest
 *     power of two >= 256 keeping at least half of each block;
 *   - otherwise the channel's DMs, sorted, are cut into classes at multiples of
 *     16 DMs, choosing the cuts and each class's N (2^8 .. 2^18) to minimise a
 *     model of device time per output sample, sum over classes of (n_dm t_inv(N)
 *     + t_fwd(N)) N / V, with t_inv and t_fwd the measured times per transform
 *     point of the inverse (per DM) and forward (per block) transforms.  Low DMs
 *     then run shorter transforms with less overlap.  Every (channel, DM)'s
 *     blocking is exported by ddx_get_layout; the visibilities of a DM depend only
 *     on its own blocking;
 * builds the FP64 tables and allocates device memory.  Returns ESTATE after the
 * first ddx_process_block, EUNSUPPORTED for N > 2^18, EINVAL if V < L. */
int ddx_set_dm_trials(ddx_plan* plan, int32_t chan, const double* dm_pc_cm3, int32_t n_dm);

/* The blocking ddx_set_dm_trials chooses for channel chan of a descriptor, computed
 * on the host alone (no plan, no device): for each of the n_dm DMs (HOST array,
 * rules as for ddx_set_dm_trials) the FFT length, kept outputs and lead of its
 * class, written to caller HOST arrays of n_dm entries.  Returns the number of
 * classes (>= 1), or EINVAL (bad descriptor or arguments, V < L) / EUNSUPPORTED
 * (N > 2^18) as ddx_set_dm_trials would. */
int ddx_plan_blocking(const ddx_desc* desc, int32_t chan, const double* dm_pc_cm3, int32_t n_dm, int32_t* fft_len,
                      int32_t* valid, int32_t* lead);

/* Restrict dedispersion and correlation of channel chan (-1 = all) to the DMs
 * with mask[d] != 0 (mask has D_c entries; NULL = all active).  Blocking is
 * unchanged, so active DMs give results bitwise equal to a full sweep.
 * Full records: inactive DMs' visibilities are written as zeros; allowed
 * between calls.  Compact records: the record holds the active (channel, DM)
 * pairs only, channel-major in DM order (record_pos in the layout); the mask
 * may change only when every dump produced so far has been fetched (ESTATE
 * otherwise), and EINVAL if more pairs than max_record_pairs would be active.
 * Host state only: no device work and no synchronisation; the next
 * ddx_process_block takes the new set. */
int ddx_set_active_dms(ddx_plan* plan, int32_t chan, const uint8_t* mask);

/* The learned proposal's selection (the proposal is this project's, not the
 * paper's): from per-DM logits d_scores[D] (DEVICE FP32, e.g. ddx_cnn_forward's
 * output) activate the k highest-scoring DMs -- ties to the lower DM index, NaN
 * lowest -- or, when more than k logits exceed logit_threshold (the proposal cannot
 * keep every candidate), every DM: the fallback to the full sweep.  The ranking
 * runs on the device in one workgroup; the mask and the fallback flag are then
 * copied to the host and hip_stream is synchronised (the next ddx_process_block
 * lists its work on the host), and the mask is applied as by ddx_set_active_dms
 * (same state rules).  chan = -1 applies one mask to every channel (all must have
 * the same D).  d_mask_out: optional DEVICE uint8 [D] that receives the mask;
 * fallback: optional host int32.  Errors: EINVAL (NULL scores, k < 1, channel out
 * of range), EUNSUPPORTED (D > 16384, or chan = -1 with differing D_c), ESTATE,
 * EDEVICE. */
int ddx_select_active_dms(ddx_plan* plan, int32_t chan, const float* d_scores, int32_t k, float logit_threshold,
                          uint8_t* d_mask_out, int32_t* fallback, void* hip_stream);

/* Export the blocking, tables and stream counters.  Pointers refer to
 * plan-owned host memory valid until the next ddx_set_dm_trials or
 * ddx_plan_destroy.  Requires ddx_set_dm_trials for every channel (ESTATE). */
int ddx_get_layout(const ddx_plan* plan, ddx_layout* out);

/* Times of dumps first_dump .. first_dump + n_dumps - 1 of channel chan at its DM
 * trial dm_index, in FP64 seconds from the stream's first sample (the bookkeeping
 * of the integrate-and-dump of Sec. 5.1 with the delay law of Eq. dmdelay).
 * Reading: sample n is taken at n / f_s and a dump stands at the mean time of its L
 * samples, t_m = (m L + (L - 1) / 2) / f_s; the dedispersed voltages are
 * index-aligned with the input, so t_m is when the dump's signal passed the channel
 * centre.  refer_infinite != 0 subtracts the centre's delay K DM / f_c^2 behind
 * infinite frequency, which puts one dispersed pulse at the same time in every
 * channel.  out: caller-owned HOST array of n_dumps doubles.  Errors: EINVAL (NULL
 * out with n_dumps > 0, chan or dm_index out of range, first_dump or n_dumps < 0),
 * ESTATE (DM trials not set). */
int ddx_dump_times(const ddx_plan* plan, int32_t chan, int32_t dm_index, int64_t first_dump, int64_t n_dumps,
                   int32_t refer_infinite, double* out);

/* Append n >= 0 samples per (channel, antenna) to the stream and enqueue all
 * work they complete on hip_stream (asynchronous).
 *   d_volts: DEVICE pointer, layout [C][M][n] samples of in_dtype, owned by the
 *            caller and valid until the stream has passed this work.
 * Block b of a class (the blocking N, V, lead of its DMs, ddx_set_dm_trials)
 * covers output samples [b V, (b+1) V) and reads input [b V - lead, b V - lead
 * + N); samples before 0 are zero.  A block runs once its whole input window has
 * arrived, and no block of a channel runs before its scale window [0, N_c -
 * lead_c) has, so results do not depend on how the stream is split into calls.  flags & DDX_FLUSH zero-pads after the
 * last sample, runs the remaining blocks and ends the stream (later calls:
 * ESTATE).  Per block and active DM d:
 *   X = DFT_N(x_b) (unnormalised, exp(-2 pi i k n / N));
 *   H[k] = exp(-2 pi i r), r = u - rint(u), u = K DM f_k^2 / (f_c^2 (f_c + f_k)),
 *     f_k = sideband * (k < N/2 ? k : k - N) f_s / N, u and r in FP64;
 *   y[b V + j] = (1/N) IDFT(X H)[lead + j], j < V;
 * and for each complete dump m (samples [m L, (m+1) L)):
 *   V_ij = sum_n y_i[n] conj(y_j[n])   (raw sum, input units squared; the
 *   correlator works on s_c y -- rounded for F16/E4M3 -- and divides by s_c^2).
 * A trailing partial dump is dropped.
 *
 * Schedule: one call lists its work for all channels at once and copies the
 * lists to the device: the (class, block) items of the forward transforms (one
 * launch per transform length), and the units (class, active DM, block) in the
 * order transform length, class, DM group, block, DM.  Units are cut into waves
 * of wave_units (a wave holds one transform length); each wave is one chirp
 * launch, one dedispersion launch (two for N > 2^15) and one correlator launch
 * over all its units' dumps, whatever channels and DMs they belong to.
 *
 * Errors: EINVAL (n < 0, n >
 * max_block_samples, NULL volts with n > 0), ESTATE (no DM trials, stream
 * flushed), EFULL (the dump ring would overwrite unfetched dumps: fetch first),
 * EDEVICE. */
int ddx_process_block(ddx_plan* plan, const void* d_volts, int64_t n, int32_t flags, void* hip_stream);

/* Copy every dump complete in all channels and not yet fetched to out (device
 * or host memory, caller-owned), enqueued on hip_stream (a host destination is
 * complete when the stream is synchronised).  Layout: [dump][channel][dm][baseline]
 * complex64 (float re, float im); the record of one dump holds record_elems
 * values, channel c / DM d at record_pos[dm_offset[c] + d] * n_baselines (full
 * records: record_pos = dm_offset[c] + d).
 * *first_dump = absolute index of the first dump returned, *n_dumps = count.
 * If cap_bytes is too small returns ESIZE with *n_dumps = the count required
 * and copies nothing.  out may be NULL when no dump is ready. */
int ddx_fetch_visibilities(ddx_plan* plan, void* out, size_t cap_bytes, int64_t* first_dump,
                           int64_t* n_dumps, void* hip_stream);

/* Start a new stream on the same plan: sample and dump counters, input history
 * and unfetched dumps are discarded; DM trials, blocking, tables and device
 * memory are kept.  Synchronises the plan's last stream first.  ESTATE before
 * ddx_set_dm_trials. */
int ddx_reset_stream(ddx_plan* plan);

/* Kernel kinds timed by the profiler. */
#define DDX_K_FORWARD 0  /* overlap-save gather + forward FFT */
#define DDX_K_CHIRP 1    /* chirp table from the FP64 phase */
#define DDX_K_DEDISP 2   /* chirp multiply + inverse FFT + discard (+ quantise) */
#define DDX_K_CORR 3     /* cross-multiply + integrate-and-dump on MFMA */
#define DDX_K_OTHER 4    /* history carry, zeroing of inactive DMs */
#define DDX_N_KINDS 5

typedef struct ddx_profile {
  int64_t launches[DDX_N_KINDS];  /* kernel launches recorded per kind */
  double time_ms[DDX_N_KINDS];    /* summed device time between the events around each launch */
  double flops[DDX_N_KINDS];      /* algorithmic flops: 5 N log2 N per FFT, 6 N per chirp multiply,
                                     8 L per baseline (i <= j) per dump */
  double bytes[DDX_N_KINDS];      /* bytes as staged through memory: forward = input + spectra;
                                     dedispersion = one spectrum read per (DM, block, antenna),
                                     one chirp per wave, the dedispersed voltages written;
                                     correlator = its dumps' voltages read + visibilities */
} ddx_profile;

/* on != 0: record a pair of hipEvents around every kernel launch on the
 * launch's stream (adds a little host overhead); on = 0 stops recording.
 * Turning it on clears earlier records. */
int ddx_set_profiling(ddx_plan* plan, int32_t on);

/* Synchronise the recorded events and sum them per kernel kind into *out. */
int ddx_get_profile(ddx_plan* plan, ddx_profile* out);

/* ---- Learned DM proposal -------------------------------------------------------
 *
 * DM-time power tiles: the paper's incoherent dedispersion (Sec. 2.3.1: detect,
 * integrate, delay each channel by the trial DM's delay, sum the channels) of
 * power beams (Sec. 2.4.1: detected power summed over antennas), for the plan's
 * trial DMs (every channel must have the same list) and its exported channel
 * shifts (samples behind the highest channel).  With p_c[n] = sum_p |x_{c,p}[n]|^2,
 *   T[d][t] = C B * sum_c sum_{n in W} p_c[n] / |W|,
 *   W = [t B + shift[c][d], (t + 1) B + shift[c][d]) clipped to the stream,
 * i.e. the mean power over the samples that exist, scaled to a full bin of B =
 * bin_len samples.  Output [D][n_bins] FP32 in caller-owned device memory. */

/* Tile of one whole stream d_volts [C][M][n] (device, in the plan's input format).
 * Errors: ESTATE (no DM trials), EUNSUPPORTED (DM lists differ between channels),
 * EINVAL, ENOMEM (plan scratch: C n floats + C (n + 1) doubles), EDEVICE. */
int ddx_power_tile(ddx_plan* plan, const void* d_volts, int64_t n, int32_t bin_len, int32_t n_bins, float* d_tile,
                   void* hip_stream);

/* The same tiles for n_tiles streams given as power already summed over antennas
 * and over fine bins of `fine` samples: d_power [n_tiles][C][units] FP32 (device).
 * Shifts are rounded to whole fine bins; bin_len must be a multiple of fine.
 * Output [n_tiles][D][n_bins].  n_tiles x C <= 65535 and D <= 65535 (EINVAL /
 * EUNSUPPORTED otherwise). */
int ddx_power_tile_from_power(ddx_plan* plan, const float* d_power, int32_t n_tiles, int64_t units, int32_t fine,
                              int32_t bin_len, int32_t n_bins, float* d_tiles, void* hip_stream);

/* A 1-D CNN that scores every DM row of a tile.  Each tile is standardised
 * ((T - mean) / std over the tile); row d's input is rows d-1, d, d+1 (edges
 * repeated) over the n_bins time bins; four convolutions (kernel 9, zero padding
 * 4, 32 channels, strides 1, 2, 2, 2, ReLU), a maximum over time and a linear
 * layer give one logit per row.  Parameters: one FP32 vector of
 * ddx_cnn_num_params values, in the order W1 [32][3][9], b1 [32], W2 [32][32][9],
 * b2, W3, b3, W4, b4, w5 [32], b5 [1].  Training minimises the mean logistic loss
 * of the row logits with Adam.  A network is not thread-safe; it holds the
 * activations of its last forward pass, and the tiles and scores buffers passed
 * to ddx_cnn_forward must stay valid until ddx_cnn_backward has run (the loss
 * reads the scores, the backward pass the tiles). */
typedef struct ddx_cnn ddx_cnn;

int ddx_cnn_num_params(int64_t* n_params);

/* Allocate a network for tiles of n_dm rows and n_bins bins (a multiple of 64),
 * at most max_tiles per call, n_dm * max_tiles <= 65535 rows (DDX_EINVAL
 * otherwise).  Parameters start at zero: set them. */
int ddx_cnn_create(int32_t n_dm, int32_t n_bins, int32_t max_tiles, ddx_cnn** out);

/* Copy parameters from host memory (resets the Adam state) / to host memory;
 * read the gradients of the last backward pass. */
int ddx_cnn_set_weights(ddx_cnn* net, const float* host_params, int64_t n);
int ddx_cnn_get_weights(ddx_cnn* net, float* host_params, int64_t n);
int ddx_cnn_get_grads(ddx_cnn* net, float* host_grads, int64_t n);

/* Arithmetic of the three convolutions (forward, backward data, backward weights).
 * DDX_CNN_FP32 (the default): FP32 on the vector units.  DDX_CNN_FP16: operands
 * rounded to IEEE binary16 (RNE) and multiplied on the matrix cores with FP32
 * accumulation; every operand tile (a layer's weights, a row's window of 64 to 256
 * time steps of activations or gradients) is first multiplied by a power of two that
 * puts its largest magnitude in [2^13, 2^14), undone exactly on the FP32 result.
 * Parameters, biases, pooling, the linear layer, the loss and Adam stay FP32 in
 * either form.  Changing the precision discards the last forward pass (run
 * ddx_cnn_forward again before ddx_cnn_loss / ddx_cnn_backward).  DDX_EINVAL for any
 * other value. */
#define DDX_CNN_FP32 0
#define DDX_CNN_FP16 1
int ddx_cnn_set_precision(ddx_cnn* net, int32_t precision);

/* Scores of every row of n_tiles tiles: d_tiles [n_tiles][n_dm][n_bins] (device),
 * d_scores [n_tiles * n_dm] (device).  Asynchronous on hip_stream. */
int ddx_cnn_forward(ddx_cnn* net, const float* d_tiles, int32_t n_tiles, float* d_scores, void* hip_stream);

/* Activations of layer 1..4 (after the ReLU) from the last forward pass, copied
 * to host memory: [rows][32][n_bins / 2^(layer-1)], rows = n_tiles * n_dm; count
 * must be that size (DDX_EINVAL otherwise, DDX_ESTATE before a forward pass).
 * Synchronises the device.  The pooling takes, per row and channel, the first
 * time index of layer 4's maximum. */
int ddx_cnn_get_activations(ddx_cnn* net, int32_t layer, float* host_acts, int64_t count);

/* After a forward pass: per-row logistic loss softplus(s) - y s into
 * d_loss_rows [rows] and its gradient (sigmoid(s) - y) / rows kept for backward. */
int ddx_cnn_loss(ddx_cnn* net, const float* d_labels, float* d_loss_rows, void* hip_stream);

/* Gradients of the mean loss with respect to every parameter. */
int ddx_cnn_backward(ddx_cnn* net, void* hip_stream);

/* One Adam step (Kingma & Ba 2015, bias-corrected) with the last gradients. */
int ddx_cnn_adam(ddx_cnn* net, float lr, float beta1, float beta2, float eps, void* hip_stream);

int ddx_cnn_destroy(ddx_cnn* net);
const char* ddx_cnn_last_error(const ddx_cnn* net);

/* ---- Chirpolator pre-integrator (Sec. 3.2, App. A.3) ----------------------------
 * For every antenna pair p < q (row-major: (0,1), (0,2), ..., (M-2,M-1)) of one
 * complex baseband stream s [M][n]:
 *   x_pq[n] = s_p[n] s_q[n]^*                                     (Sec. 3.2, Eq. xpq)
 *   V_k[m]  = sum_{j<L} exp(-2 pi i (j + m L) k / N) x_pq[j + m L]  (App. A.3, block partial DFT)
 *   S_k[m]  = S_k[m-1] + V_k[m] - V_k[m - N/L]                    (App. A.3, Eq. block_cic)
 * for the bins k = -kmax..kmax and the complete blocks m of the stream, from zero
 * state, so S_k[m] is bin k of the DFT of the N samples ending with block m (phase
 * referenced to sample 0).  Only complete windows are returned: m = N/L - 1 ..
 * n/L - 1.  FP32 products, FP32 sums over a block, FP64 moving sum, FP32 output.
 * One pre-integrator serves one DFT length N (one DM bank); it is not thread-safe. */
typedef struct ddx_chirp ddx_chirp;

/* n_ant in [2, 1024]; block_len L >= 1; fft_n N a multiple of L; 0 <= kmax with
 * 2 kmax + 1 <= N; max_samples >= N bounds n per call (it sizes the partial-DFT
 * workspace: (max_samples / L) (M (M-1) / 2) (2 kmax + 1) complex64).  EINVAL for
 * out-of-range arguments, ENOMEM / EDEVICE for device failures. */
int ddx_chirp_create(int32_t n_ant, int32_t fft_n, int32_t block_len, int32_t kmax, int64_t max_samples,
                     ddx_chirp** out);

/* Shape of the output of a call with n samples: *n_windows = max(0, n/L - N/L + 1)
 * complete windows, *n_pairs = M (M-1) / 2, *n_bins = 2 kmax + 1. */
int ddx_chirp_output_shape(const ddx_chirp* c, int64_t n, int64_t* n_windows, int32_t* n_pairs, int32_t* n_bins);

/* d_volts: DEVICE [M][n] complex64 (float re, float im), caller-owned; d_out:
 * DEVICE [n_windows][n_pairs][n_bins] complex64, bin index k + kmax.  Asynchronous
 * on hip_stream; the inputs must stay valid until the stream has passed the work.
 * A stream shorter than one window returns DDX_OK and writes nothing.  EINVAL for
 * n outside [0, max_samples] or a NULL buffer, EDEVICE for launch failures. */
int ddx_chirp_preintegrate(ddx_chirp* c, const void* d_volts, int64_t n, void* d_out, void* hip_stream);

/* Per-pair bin budgets (Sec. "compute only DFTs required on a baseline basis"):
 * kmax_pair [M (M-1) / 2] host array in pair order, 0 <= kmax_pair <= kmax, or NULL
 * for kmax everywhere.  Bins |k| > kmax_pair of a pair are not computed and are
 * written as zero.  Pairs are processed in descending budget order, so tiles of
 * pairs whose budgets are all below a tile of bins are skipped.  Synchronises the
 * device; EINVAL for an out-of-range budget. */
int ddx_chirp_set_pair_bins(ddx_chirp* c, const int32_t* kmax_pair);

/* Synchronises the device and frees the pre-integrator.  NULL is a no-op. */
int ddx_chirp_destroy(ddx_chirp* c);
const char* ddx_chirp_last_error(const ddx_chirp* c);

/* A bank of the same pre-integrator over the window lengths N = n0 d, d = 1 ..
 * n_len (App. A.3, a DFT length per DM trial), with the factorisation of App. A.3
 * ("Factorizing the DFTs"): a bin k that shares a factor with d is formed, for the
 * smallest prime p dividing gcd(|k|, d) (gcd(0, d) = d), as the sum of p adjacent
 * windows of bin k / p of length n0 d / p; the other bins are computed directly.
 * Constraints as for ddx_chirp_create with N = n0, plus 1 <= n_len <= 64 and
 * max_samples >= n0 n_len.  Not thread-safe. */
typedef struct ddx_chirp_bank ddx_chirp_bank;

int ddx_chirp_bank_create(int32_t n_ant, int32_t n0, int32_t n_len, int32_t block_len, int32_t kmax,
                          int64_t max_samples, ddx_chirp_bank** out);

/* Output layout of a call with n samples: length d's windows [n/L - n0 d/L + 1]
 * (or 0) x [pairs] x [2 kmax + 1] complex64 start at element offsets[d - 1];
 * windows and offsets are host arrays of n_len entries; *total = all elements. */
int ddx_chirp_bank_layout(const ddx_chirp_bank* b, int64_t n, int64_t* windows, int64_t* offsets, int64_t* total);

/* d_volts: DEVICE [M][n] complex64; d_out: DEVICE, *total complex64 in the layout
 * above.  Asynchronous on hip_stream.  Errors as for ddx_chirp_preintegrate. */
int ddx_chirp_bank_run(ddx_chirp_bank* b, const void* d_volts, int64_t n, void* d_out, void* hip_stream);

/* Per-pair bin budgets for every length of the bank, as ddx_chirp_set_pair_bins. */
int ddx_chirp_bank_set_pair_bins(ddx_chirp_bank* b, const int32_t* kmax_pair);

int ddx_chirp_bank_destroy(ddx_chirp_bank* b);
const char* ddx_chirp_bank_last_error(const ddx_chirp_bank* b);

/* ---- Post-integrator imaging (Sec. 3.3, 3.4, App. A.1) ----------------------
 * The detection image of the Chirpolator from the pre-integrator's bins: for
 * each window and each direction (l, m),
 *   P = sum_{p<q} sum_{t=-F..F} conj(Phi_pq(x)) D_N(x) / N * X_pq[k0' + t],
 *   E = |P|^2  (Eq. eth),
 * with tau_pq = (u l + v m + w (n - 1)) / c for (u, v, w) = r_p - r_q (Eq. tau3D,
 * n = sqrt(1 - l^2 - m^2), c = 299792458 m/s), k0 = fdot tau N / f_s (Eq. f0),
 * k0' = rint(k0) (ties to even, FP64), x = k0' + t - k0, D_N of Eq. dn and
 * Phi_pq(x) = exp(-pi i fdot tau (a_p + a_q)) exp(-pi i x (N - 1) / N) (Eq.
 * phipq1, with a_p = -r_p . (l, m, n - 1) / c the delay of antenna p relative to
 * the phase centre).  X_w[k] = S_w[k] exp(2 pi i w L k / N) re-references the
 * pre-integrator's window w (which starts at sample w L; its bins are phase-
 * referenced to sample 0) to its own first sample.  Bins |k| > kmax contribute
 * nothing.  Pairs p < q in row-major order, as ddx_chirp_preintegrate writes.
 * Directions are processed in tiles of 256 consecutive entries of pix_lm: list
 * neighbouring directions together (e.g. 16 x 16 blocks of a grid) so that a
 * tile reads few bins per pair. */
typedef struct ddx_image ddx_image;

/* ant_xyz: HOST [n_ant][3] antenna positions in metres (any common origin);
 * pix_lm: HOST [n_pix][2] direction cosines with l^2 + m^2 < 1; fdot_hz_s: chirp
 * rate; samp_rate_hz: f_s; fft_n: N; block_len: L (N / L <= 65535); kmax <= 640
 * with 2 kmax + 1 <= N: the bins of the input; half_width: F in 0..8.  Both host
 * arrays are read during the call only.  Computes the weights on the device
 * (synchronously) and keeps them: 8 (2F + 1) + 4 bytes per (pair, direction).
 * DDX_EINVAL for invalid arguments, DDX_ENOMEM, DDX_EDEVICE. */
int ddx_image_create(int32_t n_ant, const double* ant_xyz, int32_t n_pix, const double* pix_lm,
                     double fdot_hz_s, double samp_rate_hz, int32_t fft_n, int32_t block_len,
                     int32_t kmax, int32_t half_width, ddx_image** out);

/* Images made by a run over n_rows input rows with step w_step: ceil(n_rows / w_step). */
int ddx_image_output_count(const ddx_image* h, int64_t n_rows, int32_t w_step, int64_t* n_images);

/* d_bins: DEVICE [n_rows][pairs][2 kmax + 1] complex64, row r = pre-integrator
 * window first_window + r (a slice of ddx_chirp_preintegrate's output).  Images
 * are made for rows 0, w_step, 2 w_step, ...: d_p DEVICE [n_images][n_pix]
 * complex64 (P) and d_e DEVICE [n_images][n_pix] float (E); either may be NULL,
 * not both.  Asynchronous on hip_stream; caller-owned buffers must stay valid
 * until the stream passes this work.  n_rows = 0 is a no-op.  DDX_EINVAL for
 * negative counts, w_step < 1 or NULL buffers; DDX_EUNSUPPORTED if the grid would
 * exceed 2^31 workgroups; DDX_EDEVICE on a launch failure. */
int ddx_image_run(ddx_image* h, const void* d_bins, int64_t n_rows, int64_t first_window, int32_t w_step,
                  void* d_p, void* d_e, void* hip_stream);

/* Synchronise the device and free the plan's memory.  NULL is a no-op. */
int ddx_image_destroy(ddx_image* h);
const char* ddx_image_last_error(const ddx_image* h);

/* ---- Classical incoherent dedispersion of power beams (Sec. 2.3.1, 2.4.1) -------
 * Stateless calls; every device buffer is caller-owned and must not overlap another
 * buffer of the same call; asynchronous on hip_stream.  Power spectrograms are
 * [C][n_t] FP32 rows, channel 0 the least delayed (highest frequency); samples past
 * n_t count as zero. */

/* Power beam (Sec. 2.4.1): d_power[c][t] = sum over antennas a and the n_int
 * samples n of interval t of |x_{c,a}[n]|^2, t < floor(n_samp / n_int).
 * d_volts: DEVICE [n_chan][n_ant][n_samp] complex64.  DDX_EINVAL for invalid
 * sizes (n_chan <= 65535) or NULL buffers. */
int ddx_power_beam(const void* d_volts, int32_t n_chan, int32_t n_ant, int64_t n_samp, int32_t n_int,
                   float* d_power, void* hip_stream);

/* Dispersion delays in whole samples relative to the highest channel (Eq.
 * dmdelay): delays[c][d] = rint(k_dm DM_d (f_c^-2 - f_top^-2) / t_samp_s), FP64,
 * ties to even.  chan_freq_hz [n_chan], dm [n_dm] and delays [n_chan][n_dm] are
 * HOST arrays.  DDX_EINVAL for non-positive frequencies or sample time, negative
 * or non-finite DMs; DDX_EUNSUPPORTED if a delay exceeds 2^31 - 1 samples. */
int ddx_incoherent_delays(int32_t n_chan, const double* chan_freq_hz, double t_samp_s, int32_t n_dm,
                          const double* dm, double k_dm, int32_t* delays);

/* Brute-force incoherent dedispersion (Sec. 2.3.1): d_out[d][t] = sum_c
 * d_power[c][t + d_delays[c][d]] for t < n_out (samples outside [0, n_t) count as
 * zero).  d_delays: DEVICE [n_chan][n_dm] int32; d_out: DEVICE [n_dm][n_out].
 * DDX_EINVAL for invalid sizes or NULL buffers, DDX_EUNSUPPORTED above 2097120 DMs
 * per call. */
int ddx_incoherent_dedisperse(const float* d_power, int32_t n_chan, int64_t n_t, const int32_t* d_delays,
                              int32_t n_dm, float* d_out, int64_t n_out, void* hip_stream);

/* The tree method the paper cites for incoherent dedispersion (Sec. 2.3.1, linear
 * dispersion): for n_chan = 2^k channels (1 .. 32768), d_out[j][t] (j < n_chan) is
 * the sum of the channels along sweep j, whose delay runs from 0 at channel 0 to j
 * at the last channel: log2(n_chan) merging stages, each adding sweep floor(j/2)
 * of the first half of a group to sweep floor(j/2) of its second half advanced by
 * j - floor(j/2) samples.  d_out, d_work: DEVICE [n_chan][n_t] FP32; d_work is
 * scratch (may be NULL when n_chan is 1, 2 or 32).  DDX_EINVAL otherwise. */
int ddx_tree_dedisperse(const float* d_power, int32_t n_chan, int64_t n_t, float* d_out, float* d_work,
                        void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): ddx_tree_dedisperse with
 * its workspace in a static device array of DDX_TREE_STATIC_MAX floats (64 MiB per
 * GPU, held until the process ends) instead of d_work; same kernels, same results.
 * Allocates nothing.  n_chan * n_t > DDX_TREE_STATIC_MAX: DDX_ESIZE, nothing
 * enqueued.  Every call on one GPU shares that GPU's array: calls that overlap on
 * one GPU (other streams, other threads) race.  Other errors as ddx_tree_dedisperse,
 * and DDX_EDEVICE if the array's device address cannot be found. */
#define DDX_TREE_STATIC_MAX (16 * 1024 * 1024)
int ddx_tree_dedisperse_static(const float* d_power, int32_t n_chan, int64_t n_t, float* d_out, void* hip_stream);

/* ---- The Chimageator on a uniform linear array (Sec. 4) --------------------------
 * Stateless calls; caller-owned device buffers that must not overlap; asynchronous
 * on hip_stream.  Antenna p sits at p times the spacing along the line. */

/* Pre-integrator: for every complete block m of L = block_len samples,
 *   G_l[m] = w_l / L sum_{p < M - l} sum_{n in block m} s_p[n] s_{p+l}[n]^*  (l = 1 .. M - 1;
 *            w_l = 1 / (M - l) if natural_weights, else 1: the gridding of Sec. 4),
 *   Y_k[m] = sum_l G_l[m] exp(-2 pi i k l / N_s), k < N_s  (the spatial DFT).
 * d_volts: DEVICE [n_ant][n] complex64; d_y: DEVICE [N_s][floor(n / L)] complex64
 * (bin-major: a trajectory reads along blocks).
 * 2 <= n_ant <= 257; N_s a power of two <= 1024.  DDX_EINVAL otherwise. */
int ddx_chimg_preintegrate(const void* d_volts, int32_t n_ant, int64_t n, int32_t block_len, int32_t n_s,
                           int32_t natural_weights, void* d_y, void* hip_stream);

/* Gridding of a line of antennas at arbitrary ascending positions (Sec. 4: an
 * arbitrary array interpolated onto the regular grid): pair p < q goes to cell l =
 * rint((x_q - x_p) / spacing) (ties to even) when 1 <= l <= n_cells.  HOST arrays:
 * positions [n_ant] (2 <= n_ant <= 64, strictly ascending), cell_ptr [n_cells + 1]
 * (cell l's pairs are entries cell_ptr[l - 1] .. cell_ptr[l] - 1), cell_pairs
 * [2 x n_ant (n_ant - 1) / 2] as (p, q) int32 pairs, row-major within a cell;
 * *n_pairs = the pairs kept.  DDX_EINVAL for invalid arguments. */
int ddx_chimg_cells(int32_t n_ant, const double* positions, double spacing, int32_t n_cells, int32_t* cell_ptr,
                    int32_t* cell_pairs, int32_t* n_pairs);

/* The pre-integrator over such cells, natural weights (1 / the pairs in the cell,
 * zero for an empty cell): G_l[m] = 1 / (count_l L) sum_{(p,q) in cell l} sum_{n in
 * block m} s_p[n] s_q[n]^*, Y_k[m] = sum_{l=1}^{n_cells} G_l[m] exp(-2 pi i k l /
 * N_s).  d_cell_ptr, d_cell_pairs: DEVICE copies of the arrays above (0 <= p < q <
 * n_ant); d_y: DEVICE [N_s][floor(n / L)].  For the trajectories the cells are a
 * line of n_cells + 1 elements: pass n_ant = n_cells + 1 there.  2 <= n_ant <= 64,
 * n_cells <= 1024, N_s a power of two <= 1024; DDX_EINVAL otherwise. */
int ddx_chimg_preintegrate_cells(const void* d_volts, int32_t n_ant, int64_t n, int32_t block_len, int32_t n_s,
                                 int32_t n_cells, const int32_t* d_cell_ptr, const int32_t* d_cell_pairs, void* d_y,
                                 void* hip_stream);

/* Trajectory sums (Eq. chimg_pth) for trials i (end bin k_end[i], duration
 * t_blocks[i] blocks) from every start block m0:
 *   P[i][m0] = sum_{m=m0}^{m0+T-1} conj(Phi(x_m)) Y_{k_m}[m],
 *   k0 = k_end ((m - m0) L + (L - 1) / 2) / (T L)  (the block average at its mean
 *   sample), k_m = rint(k0) mod N_s (FP64, ties to even), x_m = k0 - rint(k0),
 *   Phi(x) = exp(pi i M x / N_s);
 * zero where m0 + T > n_blocks.  d_y as written by ddx_chimg_preintegrate; d_k_end
 * (double) and d_t_blocks (int32): DEVICE [n_trials]; d_p: DEVICE [n_trials]
 * [n_blocks] complex64.  DDX_EINVAL for invalid sizes or NULL buffers,
 * DDX_EUNSUPPORTED above 65535 trials per call. */
int ddx_chimg_trajectories(const void* d_y, int64_t n_blocks, int32_t n_ant, int32_t n_s, int32_t block_len,
                           const double* d_k_end, const int32_t* d_t_blocks, int32_t n_trials, void* d_p,
                           void* hip_stream);

/* Trajectories of a common gradient (App. B, optimising the imaging step): for
 * gradients g_i (bins per block) and durations lengths[j] (blocks, ascending, >= 1),
 *   P[i][j][m0] = sum_{q < lengths[j]} conj(Phi(x_q)) Y_{k_q}[m0 + q],
 *   k0(q) = g_i (q L + (L - 1) / 2) / L, k_q = rint(k0) mod N_s (FP64, ties to even),
 * i.e. the trajectory that ends at bin g_i lengths[j] after lengths[j] blocks; every
 * duration is a partial sum of one pass along the line.  Zero where m0 + lengths[j]
 * > n_blocks.  d_grad (double) [n_grad], d_lengths (int32) [n_len]: DEVICE; d_p:
 * DEVICE [n_grad][n_len][n_blocks] complex64.  Durations out of order leave their
 * outputs unwritten.  Errors as for ddx_chimg_trajectories. */
int ddx_chimg_gradient_sums(const void* d_y, int64_t n_blocks, int32_t n_ant, int32_t n_s, int32_t block_len,
                            const double* d_grad, int32_t n_grad, const int32_t* d_lengths, int32_t n_len, void* d_p,
                            void* hip_stream);

/* App. B's sampling rule: a trajectory ending at bin k_end after t_blocks blocks is
 * sampled kappa_t = max(1, |k_end| kappa_t0) times (the oversampling proportional to
 * the end bin; at least once); returns the whole blocks per integrated sample,
 * max(1, floor(t_blocks / kappa_t)) (host, FP64), or DDX_EINVAL (t_blocks < 1,
 * kappa_t0 < 0 or not finite). */
int ddx_chimg_sampling_blocks(double k_end, int32_t t_blocks, double kappa_t0);

/* App. B's widened and sampled trajectories (spectral smearing, sampling): for
 * trials i (end bin k_end[i], duration t_blocks[i] blocks, a_i = d_a_blocks[i] blocks
 * per integrated sample, or 1 for all when d_a_blocks is NULL), from every start
 * block m0, over the J = floor(T / a) integrated samples j (the block average of
 * sample j stands at its mean sample, k0 = k_end (j a L + (a L - 1) / 2) / (T L), k_j
 * = rint(k0) in FP64, ties to even):
 *   half_width F = 0:  P = sum_j conj(Phi(x_j)) Y'_{k_j}[j]  (Eq. chimg_pth),
 *   F >= 1:            P = sum_j sum_{t=-F..F} conj(Phi(x)) S(x) / (M - 1) Y'_{k_j+t}[j],
 *                      x = k0 - (k_j + t), S(x) = sin(pi (M - 1) x / N_s) / sin(pi x / N_s)
 *                      (the matched filter of a spatial tone over 2F + 1 bins),
 * with Y'_k[j] = sum_{r < a} Y_k[m0 + j a + r] and bins taken mod N_s; zero where m0 +
 * T > n_blocks.  Buffers as ddx_chimg_trajectories; d_a_blocks: DEVICE int32
 * [n_trials] or NULL.  DDX_EINVAL for invalid sizes, NULL buffers or F > 16. */
int ddx_chimg_trajectories_ext(const void* d_y, int64_t n_blocks, int32_t n_ant, int32_t n_s, int32_t block_len,
                               const double* d_k_end, const int32_t* d_t_blocks, const int32_t* d_a_blocks,
                               int32_t half_width, int32_t n_trials, void* d_p, void* hip_stream);

/* Gridding of a planar array (Sec. 4 step 4; App. B's gridding): pair p < q goes to
 * the cell c = rint((r_q - r_p) / spacing) per axis (ties to even); cells are kept in
 * one half plane, cu > 0 or (cu = 0, cv > 0), a pair whose offset falls in the other
 * half being stored turned round, (q, p) in cell -c; the cell (0, 0) is dropped.
 * HOST arrays: positions [n_ant][2] (x, y) (2 <= n_ant <= 64), cell_ptr [max_cells +
 * 1], cell_pairs [2 x n_ant (n_ant - 1) / 2] as (a, b) int32 pairs (the product s_a
 * s_b^*), cell_uv [2 x max_cells] as (cu, cv).  Cells ascend in (cu, cv); each cell's
 * pairs keep the row-major order of p < q.  *n_cells, *n_pairs: the cells and pairs
 * written.  DDX_ESIZE if more than max_cells cells, DDX_EINVAL otherwise. */
int ddx_chimg_cells_2d(int32_t n_ant, const double* positions, double spacing, int32_t max_cells, int32_t* n_cells,
                       int32_t* cell_ptr, int32_t* cell_pairs, int32_t* cell_uv, int32_t* n_pairs);

/* Planar pre-integrator: per complete block m of L samples, the cells' natural-weight
 * averages G_c[m] = 1 / (count_c L) sum_{(a, b) in c} sum_{n in block m} s_a[n]
 * s_b[n]^*, then the 2-D spatial DFT
 *   Y[ku N_s + kv][m] = sum_c G_c[m] exp(-2 pi i (ku cu + kv cv) / N_s),  ku, kv < N_s.
 * Cell tables as written by ddx_chimg_cells_2d, on the DEVICE.  d_y: DEVICE [N_s^2]
 * [floor(n / L)] complex64.  2 <= n_ant <= 64, N_s a power of two <= 256, n_cells <=
 * 1024; DDX_EINVAL otherwise. */
int ddx_chimg_preintegrate_2d(const void* d_volts, int32_t n_ant, int64_t n, int32_t block_len, int32_t n_s,
                              int32_t n_cells, const int32_t* d_cell_ptr, const int32_t* d_cell_pairs,
                              const int32_t* d_cell_uv, void* d_y, void* hip_stream);

/* Planar trajectories (Eq. chimg_pth on the plane): for trials i with end bins
 * d_k_end[2 i], d_k_end[2 i + 1] (double) and durations t_blocks[i] <= max_t, from every
 * start block m0:
 *   P[i][m0] = sum_{q < T} conj(R(x_q)) / |R(x_q)| Y[bu N_s + bv][m0 + q],
 *   k0 = k_end f per axis, f = (q L + (L - 1) / 2) / (T L), (bu, bv) = rint(k0) mod N_s
 *   (FP64, ties to even), x_q = k0 - rint(k0), R(x) = sum over the occupied cells of
 *   exp(2 pi i (xu cu + xv cv) / N_s) (the cells' response to a unit tone);
 * zero where m0 + T > n_blocks.  d_table_bins (int32) and d_table_w (complex64)
 * [n_trials][max_t]: DEVICE workspace for the step tables (written, then read).
 * DDX_EINVAL for invalid sizes or NULL buffers; a trial with T > max_t gives zeros. */
int ddx_chimg_trajectories_2d(const void* d_y, int64_t n_blocks, int32_t n_s, int32_t block_len, int32_t n_cells,
                              const int32_t* d_cell_uv, const double* d_k_end, const int32_t* d_t_blocks,
                              int32_t n_trials, int32_t max_t, int32_t* d_table_bins, void* d_table_w, void* d_p,
                              void* hip_stream);

/* Synchronise the plan's last stream and free plan-owned memory.  NULL is a no-op. */
int ddx_plan_destroy(ddx_plan* plan);

/* Static description of a status code. */
const char* ddx_strerror(int status);

/* Message for the last failing call on this plan ("" if none). */
const char* ddx_last_error(const ddx_plan* plan);

#ifdef __cplusplus
}
#endif

#endif /* DDX_H */
