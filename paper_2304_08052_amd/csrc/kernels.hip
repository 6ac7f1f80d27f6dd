// gfx950 kernels of the FRAM-RIR library and their C-ABI launchers.
//
//   draw_kernel      Sec. III-B, III-C, Eq. 3, 4, 6: one thread per virtual
//                    source; Philox4x32-10 words -> FP64 draws -> image table.
//   render_kernel    Eq. 1, 8: persistent grid over work items (source,
//                    microphone group, time tile); per (image, microphone) pair
//                    an FP64 delay, then 81 windowed-sinc taps accumulated in an
//                    LDS tile as fixed-point integers (ds_add_u32) under a
//                    per-row scale that cannot overflow; coalesced writeback.
//   backward_kernel  adjoint of the render with the image table held fixed:
//                    per pair 81-tap dot products of dL/dh with P and P'.
//   finalize_kernel  fixed-order reduction of the backward partials.
//
// Compiled with -ffp-contract=off: FP64 draw arithmetic is rounded one
// operation at a time, in the order the method states.  FMAs in the render
// are written explicitly.
#include <hip/hip_runtime.h>

#include <utility>

#include "../../include/framrir.h"
#include "framrir_internal.h"
#include "plan_internal.h"
#include "tap_poly.h"

using namespace framrir;

namespace {

constexpr double kTwoPi = 6.283185307179586;    // double nearest 2 pi
constexpr double kPi = 3.141592653589793;       // double nearest pi
constexpr float kPiF = 3.14159265358979323846f;
constexpr float kInvPiF = 0.318309886183790671538f;

// ---- compile-time tap tables: cos(pi m / 81), sin(pi m / 81), m = -40..40,
// from their Taylor series in FP64 (|pi m / 81| < 1.56, 16 terms).
constexpr double ct_sin(double x) {
    double term = x, sum = x;
    for (int k = 1; k < 16; ++k) {
        term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
        sum += term;
    }
    return sum;
}
constexpr double ct_cos(double x) {
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 16; ++k) {
        term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
        sum += term;
    }
    return sum;
}
constexpr double kPiOver81 = 3.14159265358979323846 / 81.0;

// ---------------------------------------------------------------------------
// Draw stage
// ---------------------------------------------------------------------------
// Table row i of source S (Sec. III-B, III-C; Eq. 3, 4, 6): row 0 is the
// direct path, row i >= 1 the virtual source drawn from Philox counter
// (i - 1, s, 0, 0).  Returns (x, y, z, g); fills aux / words when non-null.
__device__ __forceinline__ double4 draw_row(const DescHeader* H, const SrcDesc* S, const RoomDesc* R, int i,
                                            double* __restrict__ aux, uint32_t* __restrict__ words) {
    const int64_t row = S->img_off + i;
    if (i == 0) {   // direct path: the source itself, no reflection (Sec. III-D)
        if (aux) {
            for (int k = 0; k < 8; ++k) aux[8 * row + k] = 0.0;
            aux[8 * row + 4] = 1.0;
            aux[8 * row + 5] = S->d0;
        }
        if (words)
            for (int k = 0; k < 4; ++k) words[4 * row + k] = 0u;
        return make_double4(S->pos[0], S->pos[1], S->pos[2], 0.0);
    }
    uint32_t x[4] = {static_cast<uint32_t>(i - 1), static_cast<uint32_t>(S->s_local), 0u, 0u};
    philox4x32_10(x, S->key0, S->key1);
    const double two_m32 = 2.3283064365386963e-10;   // 2^-32
    const double u0 = (static_cast<double>(x[0]) + 0.5) * two_m32;
    const double u1 = (static_cast<double>(x[1]) + 0.5) * two_m32;
    const double u2 = (static_cast<double>(x[2]) + 0.5) * two_m32;
    const double u3 = (static_cast<double>(x[3]) + 0.5) * two_m32;
    const double theta = u0 * kTwoPi;                          // azimuth ~ U[0, 2 pi]
    const double phi = (u1 - 0.5) * kPi;                       // elevation ~ U[-pi/2, pi/2]
    const double arg = H->a3 + u2 * (H->b3 - H->a3);           // inverse CDF of Eq. 3
    const double xhat = cbrt_rn(arg);
    const double p = H->a + u3 * H->b_minus_a;                 // p ~ U(a, b)
    const double tt = (xhat - H->alpha) / H->beta_minus_alpha;
    const double dr = 1.0 + tt * (S->q - 1.0);                 // Eq. 4
    const double dist = S->d0 * dr;                            // D = d0 DR
    const double s2 = dist / S->ct;
    double g = 1.0 + (s2 * s2) * (S->rrmax - 1.0);             // Eq. 6
    double drt;
    if (H->tau_code == kTauQuarter) drt = sqrt_rn(sqrt_rn(dr));
    else if (H->tau_code == kTauHalf) drt = sqrt_rn(dr);
    else drt = dr;
    g = g + p * drt;
    g = fmin(fmax(g, 1.0), S->rrmax);
    // cos and sin of theta = 2 pi u0 and phi = pi (u1 - 1/2) from the exact
    // arguments 2 u0 and u1 - 1/2
    double st, ctheta, sp, cp;
    sincospi_d(2.0 * u0, &st, &ctheta);
    sincospi_d(u1 - 0.5, &sp, &cp);
    if (aux) {
        double* a = aux + 8 * row;
        a[0] = theta;
        a[1] = phi;
        a[2] = xhat;
        a[3] = p;
        a[4] = dr;
        a[5] = dist;
        a[6] = g;
        a[7] = 0.0;
    }
    if (words)
        for (int k = 0; k < 4; ++k) words[4 * row + k] = x[k];
    return make_double4(R->centre[0] + dist * (cp * ctheta), R->centre[1] + dist * (cp * st),
                        R->centre[2] + dist * sp, g);
}

__global__ void __launch_bounds__(256) draw_kernel(const void* __restrict__ desc, double* __restrict__ table,
                                                   double* __restrict__ aux, uint32_t* __restrict__ words) {
    const DescHeader* H = hdr(desc);
    const int s = blockIdx.y;
    if (s >= H->n_src) return;
    const SrcDesc* S = srcs(desc) + s;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S->n_img) return;
    const RoomDesc* R = rooms(desc) + S->room;
    *reinterpret_cast<double4*>(table + 4 * (S->img_off + i)) = draw_row(H, S, R, i, aux, words);
}

// ---------------------------------------------------------------------------
// Per-pair setup shared by the render and the adjoint
// ---------------------------------------------------------------------------
struct Pair {
    int k;        // tap centre floor(t + 1/2)
    float dl;     // fractional delay t - k in [-1/2, 1/2]
    float A;      // r^g / D
    float S;      // A sin(pi dl) / pi
    float cy, sy; // cos, sin of pi dl / 81
    float sinc;   // sin(pi dl) / (pi dl), 1 at 0
    float ux, uy, uz, D;
};

// sinc(x) = sin(pi x) / (pi x) for |x| <= 1/2 from its Taylor series in
// z = (pi x)^2 (terms to z^6; the first omitted term is below 5e-10).
__device__ __forceinline__ float sinc_small(float x) {
    const float px = kPiF * x;
    const float z = px * px;
    float acc = 1.0f / 6227020800.0f;                   // 1/13!
    acc = __builtin_fmaf(acc, z, -1.0f / 39916800.0f);  // 1/11!
    acc = __builtin_fmaf(acc, z, 1.0f / 362880.0f);     // 1/9!
    acc = __builtin_fmaf(acc, z, -1.0f / 5040.0f);      // 1/7!
    acc = __builtin_fmaf(acc, z, 1.0f / 120.0f);        // 1/5!
    acc = __builtin_fmaf(acc, z, -1.0f / 6.0f);         // 1/3!
    return __builtin_fmaf(acc, z, 1.0f);
}

// Per-pair setup: D = |pos - mic| and t = D fs / c in FP64 (delays up to
// ~6e4 samples must stay accurate to ~1e-7 samples), then FP32 quantities.
__device__ __forceinline__ Pair pair_setup(double px, double py, double pz, double mx, double my, double mz,
                                           double fs_over_c, float amp) {
    Pair P;
    const double dx = px - mx, dy = py - my, dz = pz - mz;
    const double d2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
    // sqrt from the hardware reciprocal square root and one Newton step
    const double rs = __builtin_amdgcn_rsq(d2);
    const double y0 = d2 * rs;
    const double D = __builtin_fma(__builtin_fma(-y0, y0, d2), 0.5 * rs, y0);
    const double t = D * fs_over_c;
    const double kf = __builtin_floor(t + 0.5);
    P.k = static_cast<int>(kf);
    P.dl = static_cast<float>(t - kf);
    const float Df = static_cast<float>(D);
    const float invD = __builtin_amdgcn_rcpf(Df);
    P.A = amp * invD;
    P.D = Df;
    P.ux = static_cast<float>(dx) * invD;
    P.uy = static_cast<float>(dy) * invD;
    P.uz = static_cast<float>(dz) * invD;
    P.sinc = sinc_small(P.dl);
    P.S = (P.A * P.dl) * P.sinc;                       // A sin(pi dl) / pi
    const float y = (kPiF / 81.0f) * P.dl;
    const float y2 = y * y;
    // |y| <= pi / 162: three Taylor terms are exact to FP32 rounding
    P.cy = __builtin_fmaf(y2, __builtin_fmaf(y2, 1.0f / 24.0f, -0.5f), 1.0f);
    P.sy = y * __builtin_fmaf(y2, __builtin_fmaf(y2, 1.0f / 120.0f, -1.0f / 6.0f), 1.0f);
    return P;
}

// ---- forward taps.  With m = j - 40 and S = A sin(pi dl) / pi,
//   A P(m - dl) = S Q_m(dl),  Q_m(dl) = (-1)^(m+1) cos^2(pi (m - dl)/81) / (m - dl).
// For |m| >= 3, Q_m is a short polynomial in dl (tap_poly.h); the taps next to
// the centre keep the quotient, with cos(pi (m - dl)/81) from the angle-sum
// identity; m = 0 is A sinc(dl) cos^2(pi dl/81), computed per pair.  Values
// arrive pre-scaled to fixed point; +1/2 and floor round them to integers.
// The tile accumulates them with ds_add_u32: gfx950 runs LDS integer atomics
// ~20x faster than FP32 ones, and integer sums do not depend on the order of
// the additions, so the output is bitwise reproducible.
template <int J, int K>
__device__ __forceinline__ float tap_horner(float dl) {
    constexpr float c = kPolyCoef[J][K];
    if constexpr (K == kPolyDeg[J]) {
        return c;
    } else {
        return __builtin_fmaf(tap_horner<J, K + 1>(dl), dl, c);
    }
}

// floor(v) as int32 in one VOP1 instruction (register operands only).
__device__ __forceinline__ int cvt_floor_i32(float v) {
    int q;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(q) : "v"(v));
    return q;
}

// Fixed-point tap value plus 1/2 (the caller floors it: round to nearest).
template <int J>
__device__ __forceinline__ float tap_value_half(float dl, float S, float cy, float sy, float v0h) {
    constexpr int m = J - kHalf;
    if constexpr (m == 0) {
        return v0h;
    } else if constexpr (kPolyDeg[J] < 0) {
        constexpr float M = static_cast<float>(m);
        constexpr float C = static_cast<float>(ct_cos(kPiOver81 * m));
        constexpr float Sn = static_cast<float>(ct_sin(kPiOver81 * m));
        constexpr float sgn = (m & 1) ? 1.0f : -1.0f;       // (-1)^(m+1)
        const float rx = __builtin_amdgcn_rcpf(M - dl);
        const float cw = __builtin_fmaf(C, cy, Sn * sy);
        return __builtin_fmaf(S, (sgn * (cw * cw)) * rx, 0.5f);
    } else {
        return __builtin_fmaf(S, tap_horner<J, 0>(dl), 0.5f);
    }
}

template <int J>
__device__ __forceinline__ void fwd_tap(int* __restrict__ row, float dl, float S, float cy, float sy, float v0h) {
    atomicAdd(row + J, cvt_floor_i32(tap_value_half<J>(dl, S, cy, sy, v0h)));
}

template <int... J>
__device__ __forceinline__ void fwd_taps(std::integer_sequence<int, J...>, int* __restrict__ row, float dl, float S,
                                         float cy, float sy, float v0) {
    (fwd_tap<J>(row, dl, S, cy, sy, v0), ...);
}

// ---- backward taps: s0 += G A P(x), s1 += G A P'(x), x = m - dl.  With
// v(dl) = A P(m - dl) = S Q_m(dl) and dS/ddl = A cos(pi dl) = Ac,
//   A P'(m - dl) = -dv/ddl = -(Ac Q_m + S Q_m').
// Q_m' comes from the derivative of the same polynomial; the taps next to the
// centre use the closed form
//   A P'(x) = (1/x) [(-1)^m (A cos(pi dl) w + (2 pi/81) S sw cw) - A P(x)],
//   w = cw^2, cw = cos(pi x/81), sw = sin(pi x/81).
template <int J, int K>
__device__ __forceinline__ float tap_horner_deriv(float dl) {
    constexpr float c = static_cast<float>((K + 1) * static_cast<double>(kPolyCoef[J][K + 1]));
    if constexpr (K + 1 == kPolyDeg[J]) {
        return c;
    } else {
        return __builtin_fmaf(tap_horner_deriv<J, K + 1>(dl), dl, c);
    }
}

template <int J>
__device__ __forceinline__ void bwd_tap(const float* __restrict__ row, float cy, float sy, float dl, float S,
                                        float Ac, float S2, float v0, float dp0, float& s0, float& s1) {
    constexpr int m = J - kHalf;
    const float G = row[J];
    if constexpr (m == 0) {
        s0 = __builtin_fmaf(G, v0, s0);
        s1 = __builtin_fmaf(G, dp0, s1);
    } else if constexpr (kPolyDeg[J] < 0) {
        constexpr float M = static_cast<float>(m);
        constexpr float C = static_cast<float>(ct_cos(kPiOver81 * m));
        constexpr float Sn = static_cast<float>(ct_sin(kPiOver81 * m));
        constexpr float sgn = (m & 1) ? -1.0f : 1.0f;   // (-1)^m
        const float rx = __builtin_amdgcn_rcpf(M - dl);
        const float cw = __builtin_fmaf(C, cy, Sn * sy);
        const float sw = __builtin_fmaf(Sn, cy, -(C * sy));
        const float w = cw * cw;
        const float val = (-sgn * S) * w * rx;
        const float inner = __builtin_fmaf(Ac, w, S2 * (sw * cw));
        const float dp = rx * __builtin_fmaf(sgn, inner, -val);
        s0 = __builtin_fmaf(G, val, s0);
        s1 = __builtin_fmaf(G, dp, s1);
    } else {
        const float q = tap_horner<J, 0>(dl);
        const float dq = tap_horner_deriv<J, 0>(dl);
        s0 = __builtin_fmaf(G, S * q, s0);
        s1 = __builtin_fmaf(-G, __builtin_fmaf(Ac, q, S * dq), s1);
    }
}

template <int... J>
__device__ __forceinline__ void bwd_taps(std::integer_sequence<int, J...>, const float* __restrict__ row, float cy,
                                         float sy, float dl, float S, float Ac, float S2, float v0, float dp0,
                                         float& s0, float& s1) {
    (bwd_tap<J>(row, cy, sy, dl, S, Ac, S2, v0, dp0, s0, s1), ...);
}

// cos(pi x) for |x| <= 1/2 from its Taylor series in z = (pi x)^2 (to z^8).
__device__ __forceinline__ float cospi_small(float x) {
    const float px = kPiF * x;
    const float z = px * px;
    float acc = 1.0f / 20922789888000.0f;                // 1/16!
    acc = __builtin_fmaf(acc, z, -1.0f / 87178291200.0f); // 1/14!
    acc = __builtin_fmaf(acc, z, 1.0f / 479001600.0f);    // 1/12!
    acc = __builtin_fmaf(acc, z, -1.0f / 3628800.0f);     // 1/10!
    acc = __builtin_fmaf(acc, z, 1.0f / 40320.0f);        // 1/8!
    acc = __builtin_fmaf(acc, z, -1.0f / 720.0f);         // 1/6!
    acc = __builtin_fmaf(acc, z, 1.0f / 24.0f);           // 1/4!
    acc = __builtin_fmaf(acc, z, -0.5f);                  // 1/2!
    return __builtin_fmaf(acc, z, 1.0f);
}

// sinc'(x) for |x| <= 1/2 from its Taylor series (no cancellation near 0):
//   sinc'(x) = sum_{k>=1} (-1)^k 2k pi^(2k) x^(2k-1) / (2k+1)!
__device__ __forceinline__ float dsinc_small(float x) {
    const float z = kPiF * kPiF * x * x;
    // coefficients (-1)^k 2k / (2k+1)! for k = 1..8, Horner in z
    float acc = 16.0f / 355687428096000.0f;
    acc = __builtin_fmaf(acc, z, -14.0f / 1307674368000.0f);
    acc = __builtin_fmaf(acc, z, 12.0f / 6227020800.0f);
    acc = __builtin_fmaf(acc, z, -10.0f / 39916800.0f);
    acc = __builtin_fmaf(acc, z, 8.0f / 362880.0f);
    acc = __builtin_fmaf(acc, z, -6.0f / 5040.0f);
    acc = __builtin_fmaf(acc, z, 4.0f / 120.0f);
    acc = __builtin_fmaf(acc, z, -2.0f / 6.0f);
    return acc * (kPiF * kPiF * x);
}

struct ItemCtx {
    WorkItem w;
    int room, s_local, T, n_mic_room, mic0_glob, n_img, rowlen;
    int64_t out_off, img_off;
    double fs_over_c, cx, cy, cz;
    double r, log2r;
    float margin;   // max |mic - centre| fs / c + 2 samples, for the tile test
    float rho;      // max |mic - centre| of the group (metres)
};

__device__ __forceinline__ void load_item(const void* desc, int item, const double* __restrict__ mic,
                                          const double* __restrict__ r_in, ItemCtx& c) {
    c.w = items(desc)[item];
    const SrcDesc* S = srcs(desc) + c.w.src;
    const RoomDesc* R = rooms(desc) + S->room;
    c.room = S->room;
    c.s_local = S->s_local;
    c.T = R->T;
    c.n_mic_room = R->n_mic;
    c.mic0_glob = R->mic0 + c.w.mic0;
    c.n_img = S->n_img;
    c.img_off = S->img_off;
    c.out_off = R->out_off;
    c.fs_over_c = R->fs_over_c;
    c.cx = R->centre[0];
    c.cy = R->centre[1];
    c.cz = R->centre[2];
    c.r = r_in ? r_in[S->room] : R->r;
    c.log2r = log2(c.r);
    c.rowlen = c.w.len + 2 * kHalo;
    double mx = 0.0;
    for (int m = 0; m < c.w.n_mic; ++m) {
        const double* q = mic + 3 * (c.mic0_glob + m);
        const double ex = q[0] - c.cx, ey = q[1] - c.cy, ez = q[2] - c.cz;
        mx = fmax(mx, __builtin_sqrt(ex * ex + ey * ey + ez * ez));
    }
    c.margin = static_cast<float>(mx * c.fs_over_c) + 2.0f;
    c.rho = static_cast<float>(mx) * 1.000001f + 1e-7f;
}

// Image position / reflection count of table row i (row 0 follows src).
__device__ __forceinline__ void image_row(const ItemCtx& c, int i, const double* __restrict__ table,
                                          const double* __restrict__ src, int src_glob, double& px, double& py,
                                          double& pz, double& g) {
    if (i == 0) {
        px = src[3 * src_glob + 0];
        py = src[3 * src_glob + 1];
        pz = src[3 * src_glob + 2];
        g = 0.0;
    } else {
        const double4 v = *reinterpret_cast<const double4*>(table + 4 * (c.img_off + i));
        px = v.x;
        py = v.y;
        pz = v.z;
        g = v.w;
    }
}

// Deterministic compaction of the rows [seg0, seg1) whose pulses may reach
// the tile core into list[]; returns the count.  Order: row index.
template <int NT>
__device__ int compact_rows(const ItemCtx& c, int seg0, int seg1, const double* __restrict__ table,
                            const double* __restrict__ src, int* __restrict__ list, int* __restrict__ wave_cnt) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int NW = NT / 64;
    int total = 0;
    const float lo = static_cast<float>(c.w.t0) - c.margin - 41.0f;
    const float hi = static_cast<float>(c.w.t0 + c.w.len) + c.margin + 41.0f;
    for (int base = seg0; base < seg1; base += NT) {
        const int i = base + tid;
        bool keep = false;
        if (i < seg1) {
            double px, py, pz, g;
            image_row(c, i, table, src, c.w.src, px, py, pz, g);
            const float ex = static_cast<float>(px - c.cx), ey = static_cast<float>(py - c.cy),
                        ez = static_cast<float>(pz - c.cz);
            const float tc = __builtin_sqrtf(ex * ex + ey * ey + ez * ez) * static_cast<float>(c.fs_over_c);
            keep = tc >= lo && tc < hi;
        }
        const uint64_t mask = __ballot(keep);
        const int before = __popcll(mask & ((uint64_t(1) << lane) - 1));
        if (lane == 0) wave_cnt[wave] = __popcll(mask);
        __syncthreads();
        int off = total;
        for (int k = 0; k < wave; ++k) off += wave_cnt[k];
        int sum = 0;
        for (int k = 0; k < NW; ++k) sum += wave_cnt[k];
        if (keep) list[off + before] = i;
        total += sum;
        __syncthreads();
    }
    return total;
}

// ---------------------------------------------------------------------------
// Render: fixed-point scale, preparation and the scatter kernel
// ---------------------------------------------------------------------------
// Fixed-point budget of the LDS accumulators: a bound on the sum of |tap|
// over every pair of a source bounds every sample of its RIRs, since the
// pulse never exceeds 1 in magnitude; the bound plus the per-add rounding
// slack is mapped just below 2^31.
constexpr float kFixedBudget = 2147483648.0f - 262144.0f;
constexpr float kBoundMargin = 1.0001f;

// ---------------------------------------------------------------------------
// Render preparation: one workgroup per source.
//   - the fixed-point scale of the source: budget / sum_i max_m r^g_i / D_im,
//     with D_im >= |pos_i - centre| - rho (rho = largest |mic - centre| of
//     the room), rows inside that sphere using the exact nearest microphone;
//     summed in a fixed order, so the scale is reproducible;
//   - a counting sort of the source's table rows by centre delay into
//     kBuckets buckets: bucket offsets and a permutation.  A time tile then
//     reads one contiguous range of rows, and the lanes of a wave add into
//     nearby LDS addresses.  Order inside a bucket is arbitrary: the render
//     accumulates integers, so its result does not depend on it.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float prep_key_tc(const RoomDesc* R, double px, double py, double pz, float& dc) {
    const float ex = static_cast<float>(px - R->centre[0]), ey = static_cast<float>(py - R->centre[1]),
                ez = static_cast<float>(pz - R->centre[2]);
    dc = __builtin_sqrtf(__builtin_fmaf(ex, ex, __builtin_fmaf(ey, ey, ez * ez)));
    return dc * static_cast<float>(R->fs_over_c);
}

__device__ __forceinline__ int bucket_of(float tc, float inv_w) {
    return min(kBuckets - 1, max(0, static_cast<int>(tc * inv_w)));
}

__device__ __forceinline__ float bucket_inv_width(int T) { return static_cast<float>(kBuckets) / (T + 256.0f); }

constexpr int kKeyCap = 8192;   // rows whose bucket index stays in LDS between the passes

// Row i of source s for the preparation: drawn here (and stored) when DRAW,
// else read from the table; row 0 always takes the render-time source.
template <bool DRAW>
__device__ __forceinline__ double4 prep_row(const DescHeader* H, const SrcDesc* S, const RoomDesc* R, int s, int i,
                                            double* __restrict__ table, const double* __restrict__ src,
                                            bool store) {
    double4 v;
    if constexpr (DRAW) {
        v = draw_row(H, S, R, i, nullptr, nullptr);
        if (store) *reinterpret_cast<double4*>(table + 4 * (S->img_off + i)) = v;
    } else {
        if (i != 0) v = *reinterpret_cast<const double4*>(table + 4 * (S->img_off + i));
    }
    if (i == 0) v = make_double4(src[3 * s], src[3 * s + 1], src[3 * s + 2], 0.0);
    return v;
}

template <bool DRAW>
__global__ void __launch_bounds__(1024) prep_kernel(const void* __restrict__ desc, double* __restrict__ table,
                                                    const double* __restrict__ mic, const double* __restrict__ src,
                                                    const double* __restrict__ r_in, float* __restrict__ src_scale,
                                                    int* __restrict__ bucket_off, int* __restrict__ perm) {
    constexpr int NT = 1024;
    static_assert(kBuckets == NT, "the bucket scan gives each thread one bucket");
    __shared__ int cnt[kBuckets];
    __shared__ unsigned short keys[kKeyCap];
    __shared__ float red[NT / 64];
    __shared__ int wsum[NT / 64];
    __shared__ float s_rho;
    const DescHeader* H = hdr(desc);
    const int s = blockIdx.x;
    if (s >= H->n_src) return;
    const SrcDesc* S = srcs(desc) + s;
    const RoomDesc* R = rooms(desc) + S->room;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    cnt[tid] = 0;
    if (tid == 0) s_rho = 0.0f;
    __syncthreads();
    if (tid < R->n_mic) {   // rho = largest |mic - centre| of the room (positive floats order as ints)
        const double* q = mic + 3 * (R->mic0 + tid);
        const double ex = q[0] - R->centre[0], ey = q[1] - R->centre[1], ez = q[2] - R->centre[2];
        atomicMax(reinterpret_cast<int*>(&s_rho), __float_as_int(static_cast<float>(__builtin_sqrt(ex * ex + ey * ey + ez * ez))));
    }
    const double r = r_in ? r_in[S->room] : R->r;
    const double log2r = log2(r);
    const float inv_w = bucket_inv_width(R->T);
    const int n = S->n_img;
    __syncthreads();
    const float rhof = s_rho * 1.000001f + 1e-7f;
    float bsum = 0.0f;
    for (int i = tid; i < n; i += NT) {
        const double4 v = prep_row<DRAW>(H, S, R, s, i, table, src, true);
        float dc;
        const float tc = prep_key_tc(R, v.x, v.y, v.z, dc);
        const float amp = exp2f(static_cast<float>(v.w * log2r));
        float dmin = dc * 0.999999f - rhof;
        if (dmin < 1e-3f) {
            dmin = 3.0e38f;
            for (int m = 0; m < R->n_mic; ++m) {
                const double* q = mic + 3 * (R->mic0 + m);
                const float dx = static_cast<float>(v.x - q[0]), dy = static_cast<float>(v.y - q[1]),
                            dz = static_cast<float>(v.z - q[2]);
                dmin = fminf(dmin,
                             __builtin_sqrtf(__builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz))) * 0.999999f);
            }
        }
        bsum += amp / dmin;
        const int key = bucket_of(tc, inv_w);
        if (i < kKeyCap) keys[i] = static_cast<unsigned short>(key);
        atomicAdd(&cnt[key], 1);
    }
    for (int off = 32; off > 0; off >>= 1) bsum += __shfl_xor(bsum, off);
    if (lane == 0) red[wave] = bsum;
    __syncthreads();
    // exclusive scan of the bucket counts: one bucket per thread
    const int c1 = cnt[tid];
    int incl = c1;
    for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(incl, off);
        if (lane >= off) incl += v;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int base = incl - c1;
    for (int w = 0; w < wave; ++w) base += wsum[w];
    int* bo = bucket_off + static_cast<int64_t>(s) * (kBuckets + 1);
    cnt[tid] = base;
    bo[tid] = base;
    if (tid == 0) {
        bo[kBuckets] = n;
        float b = 0.0f;
        for (int w = 0; w < NT / 64; ++w) b += red[w];
        b *= kBoundMargin;
        src_scale[s] = (b > 0.0f && b < 3.0e38f) ? kFixedBudget / b : 0.0f;
    }
    __syncthreads();
    for (int i = tid; i < n; i += NT) {
        int key;
        if (i < kKeyCap) {
            key = keys[i];
        } else {   // recompute: the same arithmetic gives the same bucket
            const double4 v = prep_row<DRAW>(H, S, R, s, i, table, src, false);
            float dc;
            key = bucket_of(prep_key_tc(R, v.x, v.y, v.z, dc), inv_w);
        }
        perm[S->img_off + atomicAdd(&cnt[key], 1)] = i;
    }
}

// ---------------------------------------------------------------------------
// Render
// ---------------------------------------------------------------------------
template <int NT, int WPE>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE)))
render_kernel(const void* __restrict__ desc, const double* __restrict__ table, const double* __restrict__ mic,
              const double* __restrict__ src, const double* __restrict__ r_in, float* __restrict__ out,
              int* __restrict__ counters, const float* __restrict__ src_scale, const int* __restrict__ bucket_off,
              const int* __restrict__ perm, int acc_words) {
    extern __shared__ int acc[];
    __shared__ double micq[3 * kMaxMicGroup];
    __shared__ int s_item;
    const DescHeader* H = hdr(desc);
    const int n_items = H->n_items;
    const int tid = threadIdx.x;
    // accumulators start at zero; each item's writeback clears what it used
    for (int k = tid; k < acc_words; k += NT) acc[k] = 0;
    for (;;) {
        if (tid == 0) s_item = atomicAdd(&counters[0], 1);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        if (item >= n_items) break;
        ItemCtx c;
        load_item(desc, item, mic, r_in, c);
        const int mg = c.w.n_mic;
        if (tid < 3 * mg) micq[tid] = mic[3 * c.mic0_glob + tid];
        const int shift = kHalo - kHalf - c.w.t0;   // LDS index of tap 0 = k + shift
        const float scale = src_scale[c.w.src];
        // rows that can reach this tile: a contiguous range of the delay order
        int lo = 0, hi = c.n_img;
        if (!c.w.full) {
            const float inv_w = bucket_inv_width(c.T);
            const int b_lo = bucket_of(c.w.t0 - c.margin - 41.0f, inv_w);
            const int b_hi = bucket_of((c.w.t0 + c.w.len + c.margin + 41.0f), inv_w);
            const int* bo = bucket_off + static_cast<int64_t>(c.w.src) * (kBuckets + 1);
            lo = bo[b_lo];
            hi = bo[b_hi + 1];
        }
        const int* rows = perm + c.img_off + lo;
        const int n_list = hi - lo;
        // The range is in delay order; visiting it as j = e * P mod n_list
        // (P prime, coprime to n_list) hands the lanes of a wave rows spread
        // over the whole range, so their LDS adds rarely meet in one word.
        int P = 97;                          // 97, 89, 83: their product exceeds any row count
        while (n_list > 0 && n_list % P == 0) P = (P == 97) ? 89 : 83;
        const int jstep = n_list > 0 ? static_cast<int>((static_cast<int64_t>(NT) * P) % n_list) : 0;
        __syncthreads();
        // ---- scatter the taps as rounded fixed-point integers.  Pair
        // p = m * n_list + e: a wave takes rows of one microphone.
        const int n_pairs = n_list * mg;
        int p = tid, m = 0, e = tid;        // (m, e) of p = tid + k NT, advanced without division
        while (e >= n_list && m < mg) {
            e -= n_list;
            ++m;
        }
        int j = n_list > 0 ? static_cast<int>((static_cast<int64_t>(e) * P) % n_list) : 0;
        double px = 0.0, py = 0.0, pz = 0.0, g = 0.0;
        if (p < n_pairs) image_row(c, rows[j], table, src, c.w.src, px, py, pz, g);
        while (p < n_pairs) {
            const int cm = m;
            const double cpx = px, cpy = py, cpz = pz, cg = g;
            p += NT;
            e += NT;
            j += jstep;
            if (j >= n_list) j -= n_list;
            while (e >= n_list && m < mg) {
                e -= n_list;
                ++m;
            }
            if (p < n_pairs)   // prefetch the next pair's row
                image_row(c, rows[j], table, src, c.w.src, px, py, pz, g);
            const float amp = exp2f(static_cast<float>(cg * c.log2r));
            const Pair P =
                pair_setup(cpx, cpy, cpz, micq[3 * cm], micq[3 * cm + 1], micq[3 * cm + 2], c.fs_over_c, amp);
            const int b0 = P.k + shift;
            if (b0 < 0 || b0 + kTaps > c.rowlen) continue;
            const float S = P.S * scale;
            const float v0h = __builtin_fmaf((P.A * scale) * P.sinc, P.cy * P.cy, 0.5f);
            fwd_taps(std::make_integer_sequence<int, kTaps>{}, acc + cm * c.rowlen + b0, P.dl, S, P.cy, P.sy, v0h);
        }
        __syncthreads();
        // writeback of the tile core, samples [t0, min(t0 + len, T)), and
        // clearing of every accumulator the item touched
        const int nvalid = min(c.w.len, c.T - c.w.t0);
        const float inv = scale > 0.0f ? 1.0f / scale : 0.0f;
        for (int mm = 0; mm < mg; ++mm) {
            float* dst = out + c.out_off + (static_cast<int64_t>(c.s_local) * c.n_mic_room + c.w.mic0 + mm) * c.T +
                         c.w.t0;
            int* row = acc + mm * c.rowlen;
            for (int k = tid; k < c.rowlen; k += NT) {
                const int v = row[k];
                if (k >= kHalo && k < kHalo + nvalid) dst[k - kHalo] = static_cast<float>(v) * inv;
                row[k] = 0;
            }
        }
        __syncthreads();
    }
    // the last workgroup to finish rewinds the queue for the next launch
    if (tid == 0) {
        __threadfence();
        const int done = atomicAdd(&counters[1], 1);
        if (done == static_cast<int>(gridDim.x) - 1) {
            atomicExch(&counters[0], 0);
            atomicExch(&counters[1], 0);
        }
    }
}

// ---------------------------------------------------------------------------
// Backward
// ---------------------------------------------------------------------------
template <int NT, int WPE>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE)))
backward_kernel(const void* __restrict__ desc, const double* __restrict__ table, const double* __restrict__ mic,
                const double* __restrict__ src, const double* __restrict__ r_in, const float* __restrict__ gout,
                float* __restrict__ partials, int* __restrict__ counters, int acc_words, int list_cap) {
    extern __shared__ float tile[];
    int* list = reinterpret_cast<int*>(tile) + acc_words;
    __shared__ int wave_cnt[NT / 64];
    __shared__ int s_item;
    const DescHeader* H = hdr(desc);
    const int n_items = H->n_items;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) s_item = atomicAdd(&counters[0], 1);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        if (item >= n_items) break;
        ItemCtx c;
        load_item(desc, item, mic, r_in, c);
        const int seg_cap = c.w.full ? c.n_img : list_cap;
        const int mg = c.w.n_mic;
        // dL/dh of the tile core; zero in the halo and beyond T, so that each
        // pair counts only the taps of this tile
        for (int m = 0; m < mg; ++m) {
            const float* g = gout + c.out_off +
                             (static_cast<int64_t>(c.s_local) * c.n_mic_room + c.w.mic0 + m) * c.T;
            for (int k = tid; k < c.rowlen; k += NT) {
                const int n = c.w.t0 - kHalo + k;
                const bool core = k >= kHalo && k < kHalo + c.w.len && n < c.T;
                tile[m * c.rowlen + k] = core ? g[n] : 0.0f;
            }
        }
        const int ipp = NT / mg;
        const int my_m = tid % mg, my_slot = tid / mg;
        const double* mq = mic + 3 * (c.mic0_glob + my_m);
        const double mx = mq[0], my = mq[1], mz = mq[2];
        const float* row = tile + my_m * c.rowlen;
        const int shift = kHalo - kHalf - c.w.t0;
        const float fsc = static_cast<float>(c.fs_over_c);
        const float inv_r = static_cast<float>(1.0 / c.r);
        float gmx = 0.f, gmy = 0.f, gmz = 0.f, gsx = 0.f, gsy = 0.f, gsz = 0.f, gr = 0.f;
        __syncthreads();
        for (int seg0 = 0; seg0 < c.n_img; seg0 += seg_cap) {
            const int seg1 = min(c.n_img, seg0 + seg_cap);
            int n_list = seg1 - seg0;
            if (!c.w.full) n_list = compact_rows<NT>(c, seg0, seg1, table, src, list, wave_cnt);
            if (my_slot < ipp) {
                for (int e = my_slot; e < n_list; e += ipp) {
                    const int i = c.w.full ? seg0 + e : list[e];
                    double px, py, pz, g;
                    image_row(c, i, table, src, c.w.src, px, py, pz, g);
                    const float amp = exp2f(static_cast<float>(g * c.log2r));
                    const Pair P = pair_setup(px, py, pz, mx, my, mz, c.fs_over_c, amp);
                    const int b0 = P.k + shift;
                    if (b0 < 0 || b0 + kTaps > c.rowlen) continue;
                    const float cpd = cospi_small(P.dl);
                    const float Ac = P.A * cpd;
                    const float S2 = (2.0f * kPiF / 81.0f) * P.S;
                    const float v0 = P.A * P.sinc * (P.cy * P.cy);
                    // A P'(-dl): sinc'(-dl) w + sinc(dl) w'(-dl), w'(-dl) = (2 pi/81) sy cy
                    const float dp0 = P.A * (-dsinc_small(P.dl) * (P.cy * P.cy) +
                                             P.sinc * (2.0f * kPiF / 81.0f) * P.sy * P.cy);
                    float s0 = 0.f, s1 = 0.f;
                    bwd_taps(std::make_integer_sequence<int, kTaps>{}, row + b0, P.cy, P.sy, P.dl, P.S, Ac, S2, v0,
                             dp0, s0, s1);
                    const float q = __builtin_fmaf(fsc, s1, s0 / P.D);
                    gmx = __builtin_fmaf(P.ux, q, gmx);
                    gmy = __builtin_fmaf(P.uy, q, gmy);
                    gmz = __builtin_fmaf(P.uz, q, gmz);
                    if (i == 0) {
                        gsx -= P.ux * q;
                        gsy -= P.uy * q;
                        gsz -= P.uz * q;
                    }
                    gr = __builtin_fmaf(static_cast<float>(g) * inv_r, s0, gr);
                }
            }
            __syncthreads();
        }
        // fixed-order reduction over the threads of each microphone
        float* red = tile;   // reuse: NT x 7 floats
        red[tid * 7 + 0] = gmx;
        red[tid * 7 + 1] = gmy;
        red[tid * 7 + 2] = gmz;
        red[tid * 7 + 3] = gsx;
        red[tid * 7 + 4] = gsy;
        red[tid * 7 + 5] = gsz;
        red[tid * 7 + 6] = gr;
        __syncthreads();
        float* part = partials + static_cast<int64_t>(item) * kPartialStride;
        if (tid < mg * 3) {
            const int m = tid / 3, k = tid % 3;
            float sum = 0.f;
            for (int t = m; t < ipp * mg; t += mg) sum += red[t * 7 + k];
            part[m * 3 + k] = sum;
        } else if (tid >= 64 && tid < 68) {
            const int k = tid - 64;   // 0..2 source, 3 r
            float sum = 0.f;
            for (int t = 0; t < ipp * mg; ++t) sum += red[t * 7 + 3 + k];
            part[3 * kMaxMicGroup + k] = sum;
        }
        __syncthreads();
    }
    if (tid == 0) {
        __threadfence();
        const int done = atomicAdd(&counters[1], 1);
        if (done == static_cast<int>(gridDim.x) - 1) {
            atomicExch(&counters[0], 0);
            atomicExch(&counters[1], 0);
        }
    }
}

// One workgroup per room: sums the partials of the room's items in the
// plan's fixed order.
__global__ void __launch_bounds__(256) finalize_kernel(const void* __restrict__ desc,
                                                        const float* __restrict__ partials,
                                                        float* __restrict__ grad_mic, float* __restrict__ grad_src,
                                                        float* __restrict__ grad_r) {
    const int b = blockIdx.x;
    const DescHeader* H = hdr(desc);
    if (b >= H->n_rooms) return;
    const RoomDesc* R = rooms(desc) + b;
    const int32_t* ri = room_items(desc) + R->item0;
    const WorkItem* it = items(desc);
    const int n_out = 3 * R->n_mic + 3 * R->n_src + 1;
    for (int o = threadIdx.x; o < n_out; o += blockDim.x) {
        float sum = 0.f;
        if (o < 3 * R->n_mic) {
            const int m = o / 3, k = o % 3;
            for (int j = 0; j < R->n_item; ++j) {
                const WorkItem& w = it[ri[j]];
                if (m >= w.mic0 && m < w.mic0 + w.n_mic)
                    sum += partials[static_cast<int64_t>(ri[j]) * kPartialStride + (m - w.mic0) * 3 + k];
            }
            if (grad_mic) grad_mic[3 * (R->mic0 + m) + k] = sum;
        } else if (o < 3 * R->n_mic + 3 * R->n_src) {
            const int s = (o - 3 * R->n_mic) / 3, k = (o - 3 * R->n_mic) % 3;
            for (int j = 0; j < R->n_item; ++j) {
                const WorkItem& w = it[ri[j]];
                if (w.src == R->src0 + s)
                    sum += partials[static_cast<int64_t>(ri[j]) * kPartialStride + 3 * kMaxMicGroup + k];
            }
            if (grad_src) grad_src[3 * (R->src0 + s) + k] = sum;
        } else {
            for (int j = 0; j < R->n_item; ++j)
                sum += partials[static_cast<int64_t>(ri[j]) * kPartialStride + 3 * kMaxMicGroup + 3];
            if (grad_r) grad_r[b] = sum;
        }
    }
}

__global__ void zero_counters_kernel(int* counters) {
    if (threadIdx.x < 2) counters[threadIdx.x] = 0;
}

__global__ void philox_kernel(const uint32_t* __restrict__ ctr, const uint32_t* __restrict__ key,
                              uint32_t* __restrict__ out, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t x[4] = {ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]};
    philox4x32_10(x, key[2 * i], key[2 * i + 1]);
    for (int k = 0; k < 4; ++k) out[4 * i + k] = x[k];
}

__global__ void cbrt_kernel(const double* __restrict__ x, double* __restrict__ y, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v = x[i];
    // positive normal arguments only (the draws never produce others)
    y[i] = (v >= 2.2250738585072014e-308 && v < __builtin_inf()) ? cbrt_rn(v)
                                                                   : (v == 0.0 ? 0.0 : __builtin_nan(""));
}

// ---------------------------------------------------------------------------
// Launch helpers
// ---------------------------------------------------------------------------
int check_launch(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fr_fail(FRAMRIR_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
    return FRAMRIR_OK;
}

bool aligned(const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" int framrir_draw(const framrir_plan* plan, const void* desc_dev, double* table_dev, double* aux_dev,
                            uint32_t* words_dev, void* stream) {
    if (!plan || !desc_dev || !table_dev) return fr_fail(FRAMRIR_E_INVALID_ARG, "plan, desc and table required");
    if (!aligned(desc_dev, 256) || !aligned(table_dev, 32))
        return fr_fail(FRAMRIR_E_INVALID_ARG, "desc must be 256-byte and table 32-byte aligned");
    const DescHeader& H = plan->header;
    const dim3 grid((H.max_img + 255) / 256, H.n_src);
    hipLaunchKernelGGL(draw_kernel, grid, dim3(256), 0, static_cast<hipStream_t>(stream), desc_dev, table_dev,
                       aux_dev, words_dev);
    return check_launch("draw_kernel");
}

namespace {

// Raises a kernel's dynamic-LDS limit to the largest budget a plan may use,
// once per kernel and process (the attribute is not a stream operation).
template <typename F>
int allow_lds(F kernel) {
    static int status = [&] {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLdsBytes);
        return e == hipSuccess ? 0 : static_cast<int>(e);
    }();
    if (status != 0)
        return fr_fail(FRAMRIR_E_DEVICE, "hipFuncSetAttribute: %s", hipGetErrorString(static_cast<hipError_t>(status)));
    return FRAMRIR_OK;
}

// Views of the render workspace (layout fixed by the plan's capacities).
struct RenderWs {
    int* counters;
    float* src_scale;
    int* bucket_off;
    int* perm;
};

RenderWs render_ws(const framrir_plan* plan, void* ws_dev) {
    char* b = static_cast<char*>(ws_dev);
    return RenderWs{reinterpret_cast<int*>(b), reinterpret_cast<float*>(b + plan->ws_scale_off),
                    reinterpret_cast<int*>(b + plan->ws_bucket_off), reinterpret_cast<int*>(b + plan->ws_perm_off)};
}

int launch_prepare(const framrir_plan* plan, const void* desc_dev, double* table_dev, const double* mic_dev,
                   const double* src_dev, const double* r_dev, void* ws_dev, hipStream_t st, bool draw) {
    const RenderWs w = render_ws(plan, ws_dev);
    // preparation (and, for the forward, the draws themselves): one workgroup per source
    if (draw)
        hipLaunchKernelGGL(prep_kernel<true>, dim3(plan->header.n_src), dim3(1024), 0, st, desc_dev, table_dev,
                           mic_dev, src_dev, r_dev, w.src_scale, w.bucket_off, w.perm);
    else
        hipLaunchKernelGGL(prep_kernel<false>, dim3(plan->header.n_src), dim3(1024), 0, st, desc_dev, table_dev,
                           mic_dev, src_dev, r_dev, w.src_scale, w.bucket_off, w.perm);
    return check_launch("prep_kernel");
}

int launch_render(const framrir_plan* plan, const void* desc_dev, const double* table_dev, const double* mic_dev,
                  const double* src_dev, const double* r_dev, float* out_dev, void* ws_dev, hipStream_t st) {
    const RenderWs w = render_ws(plan, ws_dev);
    const int lds = plan->launch.lds_bytes;
    const int acc_words = plan->launch.lds_bytes / 4;
    const dim3 grid(plan->grid), block(plan->launch.wg_threads);
    const int key = plan->launch.wg_threads * 16 + plan->launch.waves_per_simd;
    switch (key) {
#define FR_CASE(NT, WPE)                                                                                    \
    case NT * 16 + WPE:                                                                                     \
        if (int rc = allow_lds(render_kernel<NT, WPE>)) return rc;                                          \
        hipLaunchKernelGGL((render_kernel<NT, WPE>), grid, block, lds, st, desc_dev, table_dev, mic_dev,   \
                           src_dev, r_dev, out_dev, w.counters, w.src_scale, w.bucket_off, w.perm,         \
                           acc_words);                                                                      \
        break;
        FR_KERNEL_SHAPES(FR_CASE)
#undef FR_CASE
        default:
            return fr_fail(FRAMRIR_E_UNSUPPORTED, "launch shape %d threads x %d waves/SIMD not compiled",
                           plan->launch.wg_threads, plan->launch.waves_per_simd);
    }
    return check_launch("render_kernel");
}

int check_render_args(const framrir_plan* plan, const void* desc_dev, const double* table_dev, const double* mic_dev,
                      const double* src_dev, const void* out_dev, void* ws_dev, size_t ws_bytes, int64_t need) {
    if (!plan || !desc_dev || !table_dev || !mic_dev || !src_dev || !out_dev || !ws_dev)
        return fr_fail(FRAMRIR_E_INVALID_ARG, "NULL argument");
    if (!aligned(desc_dev, 256) || !aligned(table_dev, 32) || !aligned(ws_dev, 256) || !aligned(out_dev, 4))
        return fr_fail(FRAMRIR_E_INVALID_ARG, "misaligned buffer");
    if (static_cast<int64_t>(ws_bytes) < need)
        return fr_fail(FRAMRIR_E_WORKSPACE, "workspace %zu < %lld bytes", ws_bytes, static_cast<long long>(need));
    return FRAMRIR_OK;
}

}  // namespace

extern "C" int framrir_prepare(const framrir_plan* plan, const void* desc_dev, double* table_dev,
                               const double* mic_dev, const double* src_dev, const double* r_dev, int draw,
                               void* ws_dev, size_t ws_bytes, void* stream) {
    int rc = check_render_args(plan, desc_dev, table_dev, mic_dev, src_dev, table_dev, ws_dev, ws_bytes,
                               plan ? plan->ws_bytes : 0);
    if (rc) return rc;
    return launch_prepare(plan, desc_dev, table_dev, mic_dev, src_dev, r_dev, ws_dev, static_cast<hipStream_t>(stream),
                          draw != 0);
}

extern "C" int framrir_render_prepared(const framrir_plan* plan, const void* desc_dev, const double* table_dev,
                                       const double* mic_dev, const double* src_dev, const double* r_dev,
                                       float* out_dev, void* ws_dev, size_t ws_bytes, void* stream) {
    int rc = check_render_args(plan, desc_dev, table_dev, mic_dev, src_dev, out_dev, ws_dev, ws_bytes,
                               plan ? plan->ws_bytes : 0);
    if (rc) return rc;
    return launch_render(plan, desc_dev, table_dev, mic_dev, src_dev, r_dev, out_dev, ws_dev,
                         static_cast<hipStream_t>(stream));
}

extern "C" int framrir_render(const framrir_plan* plan, const void* desc_dev, const double* table_dev,
                              const double* mic_dev, const double* src_dev, const double* r_dev, float* out_dev,
                              void* ws_dev, size_t ws_bytes, void* stream) {
    int rc = framrir_prepare(plan, desc_dev, const_cast<double*>(table_dev), mic_dev, src_dev, r_dev, 0, ws_dev,
                             ws_bytes, stream);
    if (rc) return rc;
    return framrir_render_prepared(plan, desc_dev, table_dev, mic_dev, src_dev, r_dev, out_dev, ws_dev, ws_bytes,
                                   stream);
}

extern "C" int framrir_forward(const framrir_plan* plan, const void* desc_dev, double* table_dev,
                               const double* mic_dev, const double* src_dev, const double* r_dev, float* out_dev,
                               void* ws_dev, size_t ws_bytes, void* stream) {
    int rc = framrir_prepare(plan, desc_dev, table_dev, mic_dev, src_dev, r_dev, 1, ws_dev, ws_bytes, stream);
    if (rc) return rc;
    return framrir_render_prepared(plan, desc_dev, table_dev, mic_dev, src_dev, r_dev, out_dev, ws_dev, ws_bytes,
                                   stream);
}

extern "C" int framrir_render_backward(const framrir_plan* plan, const void* desc_dev, const double* table_dev,
                                       const double* mic_dev, const double* src_dev, const double* r_dev,
                                       const float* grad_out_dev, float* grad_mic_dev, float* grad_src_dev,
                                       float* grad_r_dev, void* ws_dev, size_t ws_bytes, void* stream) {
    int rc = check_render_args(plan, desc_dev, table_dev, mic_dev, src_dev, grad_out_dev, ws_dev, ws_bytes,
                               plan ? plan->ws_bwd_bytes : 0);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    int* counters = static_cast<int*>(ws_dev);
    float* partials = reinterpret_cast<float*>(static_cast<char*>(ws_dev) + kWsCounterBytes);
    const int lds = plan->launch.lds_bytes + 4 * plan->list_cap;
    const int acc_words = plan->launch.lds_bytes / 4;
    const dim3 grid(plan->grid), block(plan->launch.wg_threads);
    const int key = plan->launch.wg_threads * 16 + plan->launch.waves_per_simd;
    switch (key) {
#define FR_CASE(NT, WPE)                                                                                     \
    case NT * 16 + WPE:                                                                                      \
        if (int rc2 = allow_lds(backward_kernel<NT, WPE>)) return rc2;                                       \
        hipLaunchKernelGGL((backward_kernel<NT, WPE>), grid, block, lds, st, desc_dev, table_dev, mic_dev,  \
                           src_dev, r_dev, grad_out_dev, partials, counters, acc_words, plan->list_cap);     \
        break;
        FR_KERNEL_SHAPES(FR_CASE)
#undef FR_CASE
        default:
            return fr_fail(FRAMRIR_E_UNSUPPORTED, "launch shape not compiled");
    }
    if ((rc = check_launch("backward_kernel"))) return rc;
    hipLaunchKernelGGL(finalize_kernel, dim3(plan->header.n_rooms), dim3(256), 0, st, desc_dev, partials,
                       grad_mic_dev, grad_src_dev, grad_r_dev);
    return check_launch("finalize_kernel");
}

extern "C" int framrir_workspace_init(void* ws_dev, size_t ws_bytes, void* stream) {
    if (!ws_dev || ws_bytes < static_cast<size_t>(kWsCounterBytes) || !aligned(ws_dev, 256))
        return fr_fail(FRAMRIR_E_WORKSPACE, "workspace must be >= %lld bytes and 256-byte aligned",
                       static_cast<long long>(kWsCounterBytes));
    hipLaunchKernelGGL(zero_counters_kernel, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream),
                       static_cast<int*>(ws_dev));
    return check_launch("zero_counters_kernel");
}

extern "C" int framrir_philox4x32(const uint32_t* ctr_dev, const uint32_t* key_dev, uint32_t* out_dev, int64_t n,
                                  void* stream) {
    if (!ctr_dev || !key_dev || !out_dev || n < 0) return fr_fail(FRAMRIR_E_INVALID_ARG, "bad philox arguments");
    if (n == 0) return FRAMRIR_OK;
    hipLaunchKernelGGL(philox_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), ctr_dev, key_dev, out_dev, n);
    return check_launch("philox_kernel");
}

extern "C" int framrir_cbrt_rn(const double* x_dev, double* y_dev, int64_t n, void* stream) {
    if (!x_dev || !y_dev || n < 0) return fr_fail(FRAMRIR_E_INVALID_ARG, "bad cbrt arguments");
    if (n == 0) return FRAMRIR_OK;
    hipLaunchKernelGGL(cbrt_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), x_dev, y_dev, n);
    return check_launch("cbrt_kernel");
}
