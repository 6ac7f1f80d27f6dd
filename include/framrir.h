/*
 * framrir.h - C ABI of the MI355X (gfx950) FRAM-RIR library.
 *
 * FRAM-RIR (Luo & Gu, arXiv 2304.08052) approximates the image-source RIR of
 * Eq. 1 by sampling, per source, I virtual sources: their distance ratio from
 * the quadratic density of Eq. 3 rescaled by Eq. 4, a direction uniform in
 * azimuth and elevation (Sec. III-B), and a fractional reflection count from
 * Eq. 6.  Every (virtual source, microphone) pair then adds r^g / D times a
 * pulse at delay D fs / c0 to that microphone's RIR (Eq. 1, Eq. 8).  Here the
 * pulse is an 81-tap Hann-windowed sinc at the output rate, so delays stay
 * fractional.
 *
 * Flow
 *   1. framrir_plan_create      host only: validates the batch, computes the
 *                               per-room and per-source scalars (Eq. 2, Eq. 5,
 *                               the image counts I) and a device descriptor
 *                               blob, and splits the work into items.
 *   2. the caller copies the blob (framrir_plan_desc) to device memory.
 *   3. framrir_draw             device: one row per virtual source, the
 *                               sampled position and reflection count.
 *   4. framrir_render           device: RIRs from the image table.
 *      framrir_render_backward  device: gradients of a loss through the render,
 *                               with the image table held fixed.
 *
 * Conventions
 *   - Every function returns 0 (FRAMRIR_OK) or a negative FRAMRIR_E_* code;
 *     framrir_last_error_detail gives a message for the calling thread.  No
 *     C++ exception crosses the ABI.  On error nothing is enqueued.
 *   - Pointers named *_dev are device pointers, all others host pointers.
 *     The caller owns every buffer.  Device functions only enqueue work on
 *     the given stream (a hipStream_t passed as void*; NULL = default stream):
 *     they never synchronise, allocate or copy from the host, so they can be
 *     captured into a hipGraph.  Asynchronous faults surface at the caller's
 *     next synchronisation.
 *   - Positions, room sizes, T60, fs, c0 and r are FP64; RIRs and gradients
 *     are FP32.
 *   - Rooms are indexed b in [0, B); their sources and microphones are stored
 *     back to back: source j of room b is row src_off[b] + j of a
 *     [sum n_src, 3] array, and likewise for microphones.
 *   - Output layout ("ragged packed"): the RIRs of room b start at float
 *     offset out_off[b] and are laid out [n_src][n_mic][T_b] (row-major).
 *     Every output sample is written, so the buffer need not be cleared.
 *   - Image table: one row of 4 doubles (x, y, z, g) per virtual source,
 *     sources back to back (img_off per source).  Row 0 of every source is
 *     the direct path (position = source, g = 0, Sec. III-D); rows 1..I are
 *     the sampled virtual sources.
 */
#ifndef FRAMRIR_H
#define FRAMRIR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FRAMRIR_OK 0
#define FRAMRIR_E_INVALID_ARG (-1) /* null pointer, count <= 0, non-finite value */
#define FRAMRIR_E_GEOMETRY (-2)    /* room size <= 0, point not strictly inside, D = 0, d0 >= c0 T60 */
#define FRAMRIR_E_RANGE (-3)       /* T60, fs, c0 <= 0; r not in (0,1); parameter out of range */
#define FRAMRIR_E_WORKSPACE (-4)   /* workspace or buffer too small */
#define FRAMRIR_E_DEVICE (-5)      /* HIP error while enqueueing */
#define FRAMRIR_E_UNSUPPORTED (-6) /* device is not gfx950, or unsupported option */

/* One room (Sec. II): shoebox size, reverberation time, sample rate, sound
 * speed and the seed of its counter-based draws.  r_override: reflection
 * coefficient to use instead of Eq. 2 (NaN = Eq. 2 as printed). */
typedef struct framrir_room {
    double size[3];    /* Lx, Ly, Lz in metres, > 0 */
    double rt60;       /* T60 in seconds, > 0 */
    double fs;         /* output sample rate in Hz, > 0 */
    double c;          /* sound speed c0 in m/s, > 0 */
    double r_override; /* NaN, or r in (0, 1) */
    uint64_t seed;     /* Philox key: (seed & 0xffffffff, seed >> 32) */
    int32_t n_src;     /* >= 1 */
    int32_t n_mic;     /* >= 1, <= FRAMRIR_MAX_MICS */
} framrir_room;

#define FRAMRIR_MAX_MICS 64
#define FRAMRIR_TAPS 81

/* Free constants of the method, which the paper names but does not fix:
 * alpha, beta of Eq. 3 (0 <= alpha < beta <= 1), a <= b of the perturbation
 * p ~ U(a, b) in Eq. 6, tau of Eq. 6 (0.25, 0.5 or 1), and the range of the
 * per-source image count I ~ U_int[img_lo, img_hi] (0 <= img_lo <= img_hi
 * <= 65535).  taps must be 81.  flags: 0, or FRAMRIR_FLAG_MULTIRATE for a
 * plan of the paper-literal multi-rate rendering (framrir_forward_multirate). */
#define FRAMRIR_FLAG_MULTIRATE 1u
typedef struct framrir_params {
    double alpha, beta, a, b, tau;
    int32_t img_lo, img_hi;
    int32_t taps;
    uint32_t flags;
} framrir_params;

/* Launch shape of the render and backward kernels (not part of the method):
 * lds_bytes      LDS accumulator budget per workgroup, a multiple of 16 in
 *                [4096, 160000], >= 28 * the workgroup size of either kernel,
 *                and at most 163840 - the render's static LDS, which is
 *                512 + 1664 * wg_threads / 64 bytes (27136 for 1024 threads),
 * wg_threads     threads per render workgroup: 256, 512 or 1024,
 * grid_wgs       workgroups of the persistent render grid (0 = as many as fit
 *                on 256 compute units at once, capped at the number of items),
 * max_mic_group  microphones per work item, 1 .. 16 (0 = 8),
 * waves_per_simd register budget: 4 or 8 resident waves per SIMD (0 = 4),
 * bwd_wg_threads threads per backward workgroup: 0 (= wg_threads), 256, 512
 *                or 1024,
 * bwd_grid_wgs   workgroups of the persistent backward grid (0 = as many as
 *                fit, capped at the number of items).
 * render_path    0: the scatter (every pulse tap added to an LDS tile of the
 *                RIR); 1: bin moments (per pair six moments of its
 *                fractional delay added to its integer-delay bin plus its five
 *                centre taps, then the fixed pulse filter over the bins on the
 *                matrix cores; waves_per_simd must be 4); the results agree
 *                within FP32 rounding.
 * A time tile holds tile_len = floor(lds_bytes / 4 / m_group) - 160 samples
 * of m_group microphones for the scatter; for the bin moments the largest
 * tile_len = 256 n (n <= 31) with 28 m_group (R + 4 ceil(R / 32)) <= lds_bytes,
 * R = tile_len + 80; rooms whose RIR is longer are split in time.  The
 * backward runs over the same work items as the render. */
typedef struct framrir_launch {
    int32_t lds_bytes;
    int32_t wg_threads;
    int32_t grid_wgs;
    int32_t max_mic_group;
    int32_t waves_per_simd;
    int32_t bwd_wg_threads;
    int32_t bwd_grid_wgs;
    int32_t render_path;
} framrir_launch;

/* Sizes of a plan. */
typedef struct framrir_plan_info {
    int32_t n_rooms;
    int32_t n_src;         /* sum over rooms of n_src */
    int32_t n_mic;         /* sum over rooms of n_mic */
    int32_t n_items;       /* render work items */
    int64_t n_img;         /* rows of the image table: sum over sources of I + 1 */
    int64_t out_floats;    /* floats of the ragged packed output */
    int64_t desc_bytes;    /* size of the device descriptor blob */
    int64_t ws_bytes;      /* workspace for framrir_render */
    int64_t ws_bwd_bytes;  /* workspace for framrir_render_backward */
    int32_t max_T;         /* longest RIR */
    int32_t max_img;       /* largest I + 1 */
    int64_t early_floats;  /* floats of the packed early-reverberation windows (framrir_early) */
    int32_t n_chan;        /* sum over rooms of n_src * n_mic */
    int32_t multirate;     /* 1 for a FRAMRIR_FLAG_MULTIRATE plan */
    int64_t mr_floats;     /* multi-rate plans: floats of one intermediate signal at r_l fs */
    int64_t ws_mr_bytes;   /* multi-rate plans: workspace of framrir_forward_multirate */
    int64_t fir_blocks;    /* render_path 1: 256-sample blocks of the bin-moment filter per render */
} framrir_plan_info;

typedef struct framrir_plan framrir_plan; /* opaque, host memory */

/* Plans a batch (host only; Sec. II, III-A, III-C, Eq. 2, 5).
 * rooms[n_rooms]; src: [sum n_src, 3] FP64 host; mic: [sum n_mic, 3] FP64
 * host.  prm and launch may be NULL for the defaults (alpha 0.25, beta 1,
 * a -2, b 2, tau 0.25, I in [1024, 4096]; lds 131072 B, 1024 threads).
 * Per room: T = ceil(T60 fs); R = V / S; r from Eq. 2 unless overridden;
 * centre = mean microphone.  Per source: d0 = |src - centre|,
 * RR_max = max(1, (log10 c0T60 - log10 d0 - 3) / log10 r), and
 * I = img_lo + ((w * (img_hi - img_lo + 1)) >> 32) from the first Philox word
 * w of counter (0, s, 1, 0).  Errors: INVALID_ARG, GEOMETRY, RANGE.
 * On success *out owns host memory; free it with framrir_plan_destroy. */
int framrir_plan_create(const framrir_room* rooms, int32_t n_rooms, const framrir_params* prm,
                        const framrir_launch* launch, const double* src, const double* mic,
                        framrir_plan** out);
void framrir_plan_destroy(framrir_plan* plan);
int framrir_plan_get_info(const framrir_plan* plan, framrir_plan_info* info);

/* Copies per-room and per-source arrays of a plan into caller buffers (any
 * pointer may be NULL): T[n_rooms], out_off[n_rooms + 1] (out_off[n_rooms] =
 * out_floats), r[n_rooms] (the coefficient used by the draws), n_img[n_src]
 * (I + 1 rows per source), img_off[n_src + 1], rrmax[n_src], d0[n_src]. */
int framrir_plan_get_arrays(const framrir_plan* plan, int32_t* T, int64_t* out_off, double* r,
                            int32_t* n_img, int64_t* img_off, double* rrmax, double* d0);

/* Layout of the early-reverberation windows (framrir_early; Eq. 9): room b's
 * windows start at float early_off[b] (early_off[n_rooms] = early_floats) as
 * [n_src][n_mic][width[b]], width = ceil(6 fs/1000) + ceil(50 fs/1000) + 1;
 * its channels (source-major) are chan_off[b] .. chan_off[b + 1] - 1 of the
 * start array.  Any pointer may be NULL. */
int framrir_plan_get_early(const framrir_plan* plan, int64_t* early_off, int32_t* width, int32_t* chan_off);

/* Host pointer to the descriptor blob (owned by the plan, desc_bytes long),
 * to be copied to 256-byte aligned device memory before the device calls. */
const void* framrir_plan_desc(const framrir_plan* plan);

/* Draw stage (Sec. III-B, III-C; Eq. 3, 4, 6).  Fills table_dev
 * [n_img][4] FP64 with (x, y, z, g) per virtual source.  For sampled row
 * i >= 1 of source s of room b, the words (w0..w3) = Philox4x32-10 of
 * counter (i - 1, s, 0, 0) under key(seed_b) give u_k = (w_k + 1/2) 2^-32 and
 *   theta = 2 pi u0, phi = pi (u1 - 1/2),
 *   xhat  = cbrt(alpha^3 + u2 (beta^3 - alpha^3))   correctly rounded,
 *   DR = 1 + (xhat - alpha) / (beta - alpha) (c0T60/d0 - 1),  D = d0 DR,
 *   p = a + u3 (b - a),
 *   g = clamp(1 + (D / c0T60)^2 (RR_max - 1) + p DR^tau, 1, RR_max),
 *   position = centre + D (cos phi cos theta, cos phi sin theta, sin phi),
 * every FP64 step rounded separately, so g is bit-identical to a sequential
 * IEEE evaluation.  aux_dev (may be NULL): [n_img][8] FP64 debug rows
 * (theta, phi, xhat, p, DR, D, g, 0); words_dev (may be NULL): [n_img][4]
 * uint32 Philox words (zero for the direct-path row). */
int framrir_draw(const framrir_plan* plan, const void* desc_dev, double* table_dev, double* aux_dev,
                 uint32_t* words_dev, void* stream);

/* Render (Eq. 1, Eq. 8).  For every source s, microphone m and table row i:
 * D = |pos_i - mic_m|, t = D fs / c0, A = r^g_i / D, and
 *   out[n] += A * P(n - t),  n = floor(t + 1/2) - 40 .. + 40, 0 <= n < T,
 *   P(x) = sinc(x) (1 + cos(2 pi x / 81)) / 2.
 * mic_dev [n_mic][3] and src_dev [n_src][3] FP64: positions to render with
 * (row 0 of each source is taken from src_dev, the other rows from the
 * table).  r_dev [n_rooms] FP64 or NULL (= the plan's r).  out_dev:
 * out_floats FP32.  ws_dev: ws_bytes of device memory,
 * 256-byte aligned, initialised once by framrir_workspace_init (or zero
 * filled); every call leaves it initialised again.  Calls that share a
 * workspace must not overlap.  Samples are accumulated as fixed-point
 * integers under a per-row scale that bounds the row's magnitude, so the
 * result is bitwise reproducible.  Errors: INVALID_ARG, WORKSPACE, DEVICE. */
int framrir_render(const framrir_plan* plan, const void* desc_dev, const double* table_dev,
                   const double* mic_dev, const double* src_dev, const double* r_dev,
                   float* out_dev, void* ws_dev, size_t ws_bytes, void* stream);

/* Draw and render in one call (table_dev as for framrir_draw): the draws
 * run inside the preparation kernel (framrir_prepare with draw = 1), then
 * framrir_render_prepared.  table_dev may be NULL: the draws are then not
 * exported (the preparation draws each row a second time where it would
 * read the table back), and the output, the workspace's delay-ordered rows
 * and everything computed from them are the same bit for bit. */
int framrir_forward(const framrir_plan* plan, const void* desc_dev, double* table_dev,
                    const double* mic_dev, const double* src_dev, const double* r_dev,
                    float* out_dev, void* ws_dev, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid allocation):
 * framrir_forward with its workspace in a static device array of the library,
 * FRAMRIR_NOALLOC_SCRATCH_BYTES (64 MiB) per device, held by every device
 * the library runs on until the process ends (its address is looked up once
 * per device, on the first call with that device current).  Arguments, the
 * table (which may be NULL) and the outputs as for framrir_forward; the
 * caller still owns the table, positions and output.  The call allocates nothing and enqueues a
 * small kernel that clears the workspace's counters, then the preparation
 * (with the draws) and the render.  Every call on one device shares that
 * device's array, which keeps the last call's contents: calls that overlap on
 * one device (other streams, other threads, or any framrir_forward_noalloc
 * still running) race and give wrong results.  Errors: WORKSPACE when the
 * plan's ws_bytes exceeds FRAMRIR_NOALLOC_SCRATCH_BYTES (nothing enqueued:
 * use framrir_forward with a caller workspace, or split the batch),
 * UNSUPPORTED for a multi-rate plan, and as framrir_forward. */
#define FRAMRIR_NOALLOC_SCRATCH_BYTES (64ll << 20)
int framrir_forward_noalloc(const framrir_plan* plan, const void* desc_dev, double* table_dev,
                            const double* mic_dev, const double* src_dev, const double* r_dev,
                            float* out_dev, void* stream);

/* framrir_forward plus the early-reverberation windows of Eq. 9 from the
 * same pass: while the render writes each output sample it also stores the
 * samples that fall in a channel's window into early_dev (layout, window
 * rule, zeros outside [0, T) and the start indices in start_dev (may be
 * NULL) as for framrir_early, whose result this equals bit for bit).
 * early_dev: early_floats FP32.  Not for multi-rate plans (UNSUPPORTED).
 * Arguments and errors otherwise as for framrir_forward. */
int framrir_forward_early(const framrir_plan* plan, const void* desc_dev, double* table_dev,
                          const double* mic_dev, const double* src_dev, const double* r_dev, float* out_dev,
                          float* early_dev, int32_t* start_dev, void* ws_dev, size_t ws_bytes, void* stream);

/* The two halves of framrir_render.  framrir_prepare (one workgroup per
 * source) computes, into the workspace, each source's fixed-point scale (a
 * bound on the sum of its pulse amplitudes over the microphones) and a copy
 * of its rows (row 0 at src_dev's position, amplitude r^g precomputed)
 * ordered by delay; with draw != 0 it first draws the rows into table_dev
 * (as framrir_draw; table_dev may then be NULL, as for framrir_forward).
 * framrir_render_prepared then renders from the workspace alone (table_dev,
 * which may be NULL, and src_dev are not read); its workspace must hold the
 * preparation of the same plan, table, positions and r.  Arguments and
 * errors as for framrir_render. */
int framrir_prepare(const framrir_plan* plan, const void* desc_dev, double* table_dev, const double* mic_dev,
                    const double* src_dev, const double* r_dev, int draw, void* ws_dev, size_t ws_bytes,
                    void* stream);
int framrir_render_prepared(const framrir_plan* plan, const void* desc_dev, const double* table_dev,
                            const double* mic_dev, const double* src_dev, const double* r_dev, float* out_dev,
                            void* ws_dev, size_t ws_bytes, void* stream);

/* Adjoint of framrir_render with the table held fixed.  grad_out_dev: dL/dh
 * in the output layout (FP32).  With u = (pos_i - mic_m) / D,
 * S0 = sum_n dL/dh[n] P(n - t) and S1 = sum_n dL/dh[n] P'(n - t):
 *   dL/dmic_m = sum_i u (A / D S0 + A fs / c0 S1)        -> grad_mic_dev [n_mic][3]
 *   dL/dsrc_s = -(the same sum over row 0 only)          -> grad_src_dev [n_src][3]
 *   dL/dr_b   = sum_{s,m,i} (g_i / r) A S0                -> grad_r_dev [n_rooms]
 * Outputs are FP32 and fully overwritten; any may be NULL.  Sums run in a
 * fixed order, so results are bitwise reproducible.  ws_dev: ws_bwd_bytes
 * (its first ws_bytes laid out as the render workspace), initialised as for
 * framrir_render.  Runs framrir_prepare (draw = 0) into ws_dev, then
 * framrir_render_backward_prepared. */
int framrir_render_backward(const framrir_plan* plan, const void* desc_dev, const double* table_dev,
                            const double* mic_dev, const double* src_dev, const double* r_dev,
                            const float* grad_out_dev, float* grad_mic_dev, float* grad_src_dev,
                            float* grad_r_dev, void* ws_dev, size_t ws_bytes, void* stream);

/* The adjoint alone, reusing a preparation already in ws_dev (ws_bwd_bytes):
 * the one a framrir_forward / framrir_render / framrir_prepare call on the
 * same workspace left for the same plan, table, positions and r.  The
 * positions and r of that preparation are the ones differentiated; mic_dev
 * and r_dev must hold the same values.  Arguments, outputs and errors as for
 * framrir_render_backward. */
int framrir_render_backward_prepared(const framrir_plan* plan, const void* desc_dev, const double* mic_dev,
                                     const double* r_dev, const float* grad_out_dev, float* grad_mic_dev,
                                     float* grad_src_dev, float* grad_r_dev, void* ws_dev, size_t ws_bytes,
                                     void* stream);

/* Gradient through the draws: the images move with the inputs.  The
 * Philox variates of every image (direction, x-hat, p) stay fixed, while d0 =
 * |src - centre| (centre = mean of the room's microphones), RR_max (Eq. 5)
 * and through them each image's distance D_i = d0 + t_i (c0 T60 - d0) (Eq. 4,
 * t_i = (x-hat_i - alpha) / (beta - alpha)), position centre + D_i dir_i and
 * reflection count g_i = clamp(gamma_i, 1, RR_max) (Eq. 6) follow src, the
 * microphones and r.  To the terms of framrir_render_backward this adds, per
 * source s and with dL/dpos_i the image's own gradient:
 *   dL/dd0   = sum_i (dir_i . dL/dpos_i)(1 - t_i) + ln(r) A S0 dg_i/dd0,
 *   dL/dsrc_s += dL/dd0 (src_s - centre) / d0,
 *   dL/dmic_m += (sum_i dL/dpos_i - dL/dd0 (src_s - centre) / d0) / M,
 *   dL/dr_b   += sum_i ln(r) A S0 dg_i/dr,
 * with dg/dd0, dg/dr from Eq. 5-6 inside the clamp, dRR_max/dd0 and
 * dRR_max/dr on the top clamp and 0 on the bottom one.  p DR_i^tau is
 * recovered from the row's reflection count (FP32 in the prepared rows).
 * The gradient is taken where the table was drawn: table_dev must hold
 * framrir_draw's rows for this plan, and mic_dev and src_dev the positions
 * the plan was made with; r is the plan's (no override).  Outputs, workspace,
 * order of the sums and errors as for framrir_render_backward; the direct
 * path (row 0) contributes as there. */
int framrir_render_backward_draws(const framrir_plan* plan, const void* desc_dev, const double* table_dev,
                                  const double* mic_dev, const double* src_dev, const float* grad_out_dev,
                                  float* grad_mic_dev, float* grad_src_dev, float* grad_r_dev, void* ws_dev,
                                  size_t ws_bytes, void* stream);

/* framrir_render_backward_draws reusing a preparation already in ws_dev: the
 * one a framrir_forward / framrir_prepare call with r_dev = NULL left for the
 * same plan, table and the plan's own positions. */
int framrir_render_backward_draws_prepared(const framrir_plan* plan, const void* desc_dev, const double* mic_dev,
                                           const float* grad_out_dev, float* grad_mic_dev, float* grad_src_dev,
                                           float* grad_r_dev, void* ws_dev, size_t ws_bytes, void* stream);

/* Early-reverberation filter of Eq. 9, at the output rate: for every
 * (source s, mic m) channel, t0 = |src_s - mic_m| fs / c0 (FP64, correctly
 * rounded square root, then one multiply and one divide) and the window
 * n - ceil(t0) in [-ceil(6 fs/1000), ceil(50 fs/1000)] of the rendered RIR.
 * out_dev: the RIRs of framrir_render / framrir_forward for the same plan and
 * positions (FP32, packed layout).  early_dev: early_floats FP32 in the layout
 * of framrir_plan_get_early; samples of the window outside [0, T) are 0, every
 * float is written.  start_dev: n_chan int32, the output index of each
 * channel's first window sample (may be negative), or NULL.  All device
 * pointers; enqueue only.  Errors: INVALID_ARG. */
int framrir_early(const framrir_plan* plan, const void* desc_dev, const double* mic_dev, const double* src_dev,
                  const float* out_dev, float* early_dev, int32_t* start_dev, void* stream);

/* The paper-literal multi-rate rendering (Sec. II, Sec. III-D, Eq. 7-8) for a
 * plan made with FRAMRIR_FLAG_MULTIRATE: per room r_h = floor(10^6 / fs),
 * r_l = floor(sqrt(r_h)) (at most 12), L = ceil(T60 r_h fs).  Draws as
 * framrir_forward; then per (image, mic) pair q = min(ceil(D / c0 r_h fs),
 * L - 1) (D correctly rounded, FP64), the impulse r^g / D at q down-sampled to
 * r_l fs with the 81-tap Hann-windowed sinc (unit peak) into inter_dev[0 ..
 * mr_floats) (packed [S][M][T_l], T_l = ceil(T60 r_l fs)), an 80 Hz
 * second-order Butterworth high-pass from rest (bilinear, prewarped; FP64
 * recurrence, exact chunked evaluation: the output state at every 256-sample
 * chunk start is found first, then re-run from there), and the decimation by
 * r_l with the same pulse in units of fs: out_dev (out_floats FP32, packed
 * [S][M][T], T = ceil(T60 fs)).  inter_dev: mr_floats FP32; ws_dev:
 * ws_mr_bytes, initialised as for framrir_render.  Enqueue only.  Errors:
 * INVALID_ARG, WORKSPACE,
 * UNSUPPORTED (not a multi-rate plan), DEVICE. */
int framrir_forward_multirate(const framrir_plan* plan, const void* desc_dev, double* table_dev,
                              const double* mic_dev, const double* src_dev, const double* r_dev, float* inter_dev,
                              float* out_dev, void* ws_dev, size_t ws_bytes, void* stream);

/* The stages of framrir_forward_multirate after the render: the high-pass of
 * the intermediate signal inter_dev[0 .. mr_floats) (read only) and the
 * decimation into out_dev.  Arguments and errors as for
 * framrir_forward_multirate. */
int framrir_multirate_filter(const framrir_plan* plan, const void* desc_dev, float* inter_dev, float* out_dev,
                             void* ws_dev, size_t ws_bytes, void* stream);

/* ---- Spatialisation and mixing (Sec. IV-A: the on-the-fly training set-up).
 * Every room of the plan has 3 sources: speakers 0 and 1 and the noise 2.
 * Each dry signal is convolved with its rendered RIRs (the full linear
 * convolution, kept for the utterance window of n_samples samples); speaker 1
 * is scaled so that 10 log10(E0 / E1) = SIR and the noise so that
 * 10 log10(E_sp / E2) = SNR, where E_s is the energy of source s's scaled
 * images over all microphones and samples and E_sp that of the sum of the two
 * speakers' images; the mixture is the sum of the three scaled images.
 *
 *   rir_dev     the plan's forward output, packed as framrir_render writes it
 *               (for a multi-rate plan: the output at fs)
 *   sig_dev     [n_src][n_samples] FP32 dry signals, sources in plan order
 *   sir_db_dev, snr_db_dev   [n_rooms] FP32 (dB)
 *   images_dev  out: [n_chan][n_samples] scaled images, channels in plan order
 *               (per room [3][n_mic][n_samples])
 *   mix_dev     out: [n_mic total][n_samples] mixtures, microphones in plan order
 *   gains_dev   out: [n_src] the gains (1 for speaker 0; 0 for a silent source)
 *   ws_dev      workspace of framrir_spatial_workspace bytes, 256-byte aligned
 * RIRs of up to 16384 samples take one 32768-point FFT per signal block;
 * longer ones (up to 262144 samples, else FRAMRIR_E_UNSUPPORTED) are cut into
 * partitions of 16384 samples whose spectra multiply the signal's block
 * spectra delayed by one block per partition, summed in partition order
 * (uniformly partitioned overlap-save); enqueues only. */
int framrir_spatial_workspace(const framrir_plan* plan, int32_t n_samples, size_t* ws_bytes);
int framrir_spatialize(const framrir_plan* plan, const void* desc_dev, const float* rir_dev, const float* sig_dev,
                       const float* sir_db_dev, const float* snr_db_dev, int32_t n_samples, float* images_dev,
                       float* mix_dev, float* gains_dev, void* ws_dev, size_t ws_bytes, void* stream);

/* Initialises the counters at the start of a render / backward workspace
 * (enqueues one small kernel; no host synchronisation). */
int framrir_workspace_init(void* ws_dev, size_t ws_bytes, void* stream);

/* Philox4x32-10 (Salmon et al., SC'11) of n counters: ctr_dev [n][4],
 * key_dev [n][2], out_dev [n][4] (uint32, device).  Test export of the
 * generator the draw stage uses. */
int framrir_philox4x32(const uint32_t* ctr_dev, const uint32_t* key_dev, uint32_t* out_dev,
                       int64_t n, void* stream);

/* Correctly rounded cube root of n finite non-negative doubles (device
 * buffers): the inverse-CDF step of Eq. 3.  Test export. */
int framrir_cbrt_rn(const double* x_dev, double* y_dev, int64_t n, void* stream);

/* Host (CPU) builds of the same draw-stage numerics as the device code:
 * correctly rounded cube root and square root of positive normal doubles,
 * and Philox4x32-10.  Test exports for machines without a GPU; host
 * buffers. */
int framrir_host_cbrt_rn(const double* x, double* y, int64_t n);
int framrir_host_sqrt_rn(const double* x, double* y, int64_t n);
int framrir_host_philox4x32(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t n);

/* ---- Handle and launch-shape tuner.  None of this is in the paper: the
 * launch shape only decides how the batch of the problem of Sec. II (rooms,
 * T60, positions, fs, c0 -> RIRs [B][S][M][T]) is split over the GPU, never
 * what is computed.
 *
 * framrir_handle_create: a handle for device `device` (host call; the
 * device's HIP runtime state is initialised).  Errors: INVALID_ARG (no such
 * device), UNSUPPORTED when the device is not a gfx950 (the kernels are
 * built for it alone), DEVICE.  It looks up the device address of the static
 * scratch of framrir_forward_noalloc for that device, and loads the tuning
 * caches: tune_cache_paths (may be NULL) holds file paths separated by ':';
 * the first is the cache framrir_tune writes (it need not exist yet; "" for
 * none), the others read-only fallbacks; entries of earlier paths take
 * precedence.  Cache file: a JSON object mapping "arch|size class" to
 * {"launch": {field: integer, ...}, "ms": median milliseconds}.
 * framrir_handle_destroy frees the handle (the caches stay on disk). */
typedef struct framrir_handle framrir_handle;
int framrir_handle_create(int32_t device, const char* tune_cache_paths, framrir_handle** out);
void framrir_handle_destroy(framrir_handle* h);

/* 1 if a device whose HIP gcnArchName is the given string runs this
 * library (gfx950, with or without feature suffixes), else 0.  Host only. */
int framrir_arch_supported(const char* gcn_arch_name);

/* The size class of a batch, the key of the tuning caches (host only):
 * "fs=F1/F2...;mics<=M;T=lo-hi" with the distinct sample rates (integer Hz,
 * ascending), the largest microphone count, and the powers of two that
 * bracket T = ceil(T60 fs) over the rooms.  buf receives it NUL-terminated.
 * Errors: INVALID_ARG, RANGE, WORKSPACE (buf too short). */
int framrir_size_class(const framrir_room* rooms, int32_t n_rooms, char* buf, size_t n);

/* Times framrir_forward (draws, preparation and render) of the given batch
 * under each candidate launch shape on the handle's device (median of reps
 * runs after two warm-up runs, HIP events on a stream of its own) and keeps
 * the fastest as the class's entry: in the handle and, when the handle has a
 * writable cache, in that file (other entries kept).  size_class: the key
 * (NULL = framrir_size_class of the rooms).  candidates: n_candidates shapes,
 * or NULL / 0 for the library's search: the scatter (render_path 0) over LDS
 * tiles, workgroup sizes, register budgets, microphone groups and grid sizes,
 * and the bin moments (render_path 1) at several tiles.  Shapes that are not
 * valid for the batch are skipped.  A set-up call: it allocates and frees
 * device memory and synchronises; never call it under graph capture.  best
 * and best_ms (may be NULL) receive the winner.  Errors: INVALID_ARG, RANGE
 * (no valid candidate), DEVICE, and those of framrir_plan_create. */
int framrir_tune(framrir_handle* h, const framrir_room* rooms, int32_t n_rooms, const framrir_params* prm,
                 const double* src, const double* mic, const char* size_class, const framrir_launch* candidates,
                 int32_t n_candidates, int32_t reps, framrir_launch* best, double* best_ms);

/* The cached launch shape of a size class on the handle's architecture:
 * *found = 1 and *out the entry, or *found = 0 and *out the default shape
 * (lds 131072, 1024 threads, 8 microphones per item, 4 waves per SIMD,
 * scatter).  Host only.  Errors: INVALID_ARG. */
int framrir_tune_lookup(const framrir_handle* h, const char* size_class, framrir_launch* out, int32_t* found);

/* Message for the last error on the calling thread (NUL-terminated, may be
 * truncated to n bytes).  Returns the length of the full message. */
int framrir_last_error_detail(char* buf, size_t n);
const char* framrir_strerror(int code);

/* Library version, (major << 16) | minor. */
int framrir_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FRAMRIR_H */
