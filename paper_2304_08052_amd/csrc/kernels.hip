// gfx950 kernels of the FRAM-RIR library and their C-ABI launchers.
//
//   draw_kernel      Sec. III-B, III-C, Eq. 3, 4, 6: one thread per virtual
//                    source; Philox4x32-10 words -> FP64 draws -> image table.
//   prep_kernel      one workgroup per source: (optionally the draws,) the
//                    fixed-point scale and the rows sorted by delay.
//   render_kernel    Eq. 1, 8: persistent grid over work items (source,
//                    microphone group, time tile); per (image, microphone) pair
//                    an FP64 delay, then 81 windowed-sinc taps accumulated in an
//                    LDS tile as fixed-point integers (ds_add_u32) under a
//                    per-source scale that cannot overflow; coalesced writeback.
//   backward_kernel  adjoint of the render with the image table held fixed
//                    (or, DRAWS, with the images moving with the inputs):
//                    per pair 81-tap dot products of dL/dh with P and P', and
//                    the fixed-order reduction of each room's partials.
//   render_moment_kernel  the second render path: per pair six moments and
//                    five centre taps into LDS bins, then a Toeplitz FIR over
//                    the bins on the fp16 matrix cores.
//   early_kernel     Eq. 9: the early-reverberation window of each channel
//                    (the render's EARLY instances store the same windows
//                    from the writeback).
//   hp_chunk_end_kernel, hp_carry_kernel, dec_frag_kernel,
//   decimate_mfma_kernel  Sec. II, the multi-rate chain after the render:
//                    the 80 Hz high-pass's states at every 32-sample
//                    sub-chunk, then the decimation by r_l as a Toeplitz
//                    product on the matrix cores, re-running the high-pass
//                    over each tile's window.
// The spatialisation kernels are in spatial.hip.
//
// Compiled with -ffp-contract=off: FP64 draw arithmetic is rounded one
// operation at a time, in the order the method states.  FMAs in the render
// are written explicitly.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
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
__device__ __forceinline__ Pair pair_from_delay(double t, double D, double dx, double dy, double dz, float amp);

__device__ __forceinline__ Pair pair_setup(double px, double py, double pz, double mx, double my, double mz,
                                           double fs_over_c, float amp) {
    const double dx = px - mx, dy = py - my, dz = pz - mz;
    const double d2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
    // sqrt from the hardware reciprocal square root and one Newton step
    const double rs = __builtin_amdgcn_rsq(d2);
    const double y0 = d2 * rs;
    const double D = __builtin_fma(__builtin_fma(-y0, y0, d2), 0.5 * rs, y0);
    return pair_from_delay(D * fs_over_c, D, dx, dy, dz, amp);
}

// The same pair on the paper's high-rate grid (Eq. 7): q = min(ceil(D / c0 *
// r_h fs), L - 1) with D correctly rounded and one rounding per operation, so
// the integer q is the one the plain definition gives; the pulse then sits at
// t = q r_l / r_h intermediate samples (the r_h -> r_l down-sampling).
__device__ __forceinline__ Pair pair_setup_high_rate(double px, double py, double pz, double mx, double my,
                                                     double mz, double c0, double hr, double lm1, double rl,
                                                     double rh, float amp) {
    const double dx = px - mx, dy = py - my, dz = pz - mz;
    const double D = sqrt_rn(dx * dx + dy * dy + dz * dz);
    const double q = fmin(__builtin_ceil((D / c0) * hr), lm1);
    return pair_from_delay((q * rl) / rh, D, dx, dy, dz, amp);
}

__device__ __forceinline__ Pair pair_from_delay(double t, double D, double dx, double dy, double dz, float amp) {
    Pair P;
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
// identity; m = 0 is A sinc(dl) cos^2(pi dl/81), computed per pair.
// Q_{-m}(dl) = -Q_m(-dl), and the table keeps that symmetry exactly, so taps
// m and -m share one evaluation: with the even and odd parts
// Q_m = E(dl^2) + dl O(dl^2),
//   S Q_m = SE + SO,   S Q_{-m} = SO - SE,
//   SE = sum_j c_{m,2j} w_j,   SO = sum_j c_{m,2j+1} v_j,
// over per-pair powers w_j = S dl^2j, v_j = S dl^(2j+1): every coefficient is
// an immediate operand of one multiply-add, summed from the highest term down.
// Values arrive pre-scaled to fixed point; v_cvt_rpi_i32_f32 rounds them to
// integers (floor(x + 1/2)).  The tile accumulates them with ds_add_u32:
// gfx950 runs LDS integer atomics ~20x faster than FP32 ones, and integer sums
// do not depend on the order of the additions, so the output is bitwise
// reproducible.
constexpr bool taps_mirrored() {
    if (kPolyDeg[kHalf] >= 0) return false;
    for (int m = 1; m <= kHalf; ++m) {
        const int d = kPolyDeg[kHalf + m];
        if (kPolyDeg[kHalf - m] != d) return false;
        for (int k = 0; k <= d; ++k) {
            const float c = kPolyCoef[kHalf + m][k];
            if (kPolyCoef[kHalf - m][k] != ((k & 1) ? c : -c)) return false;
        }
    }
    return true;
}
static_assert(taps_mirrored(), "the forward evaluates taps m and -m together");

constexpr int poly_top() {
    int d = 0;
    for (int j = 0; j < kTaps; ++j) d = kPolyDeg[j] > d ? kPolyDeg[j] : d;
    return d;
}
constexpr int kPolyTop = poly_top();
constexpr int kPowTerms = kPolyTop / 2 + 1;   // w_j, v_j for j < kPowTerms

// sum_{j = I}^{top} c_{J, 2j + P} pw_j, highest term first
template <int J, int P, int I, int TOP>
__device__ __forceinline__ float coef_chain(const float (&pw)[kPowTerms]) {
    constexpr float c = kPolyCoef[J][2 * I + P];
    if constexpr (I == TOP) {
        return pw[I] * c;
    } else {
        return __builtin_fmaf(pw[I], c, coef_chain<J, P, I + 1, TOP>(pw));
    }
}

// Nearest integer, floor(v + 1/2), in one VOP1 instruction (register operands only).
__device__ __forceinline__ int cvt_rpi_i32(float v) {
    int q;
    asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(q) : "v"(v));
    return q;
}

// Quotient form of a tap next to the centre (|m| = 1, 2).
template <int m>
__device__ __forceinline__ float tap_quotient(float dl, float S, float cy, float sy) {
    constexpr float M = static_cast<float>(m);
    constexpr float C = static_cast<float>(ct_cos(kPiOver81 * m));
    constexpr float Sn = static_cast<float>(ct_sin(kPiOver81 * m));
    constexpr float sgn = (m & 1) ? 1.0f : -1.0f;       // (-1)^(m+1)
    const float rx = __builtin_amdgcn_rcpf(M - dl);
    const float cw = __builtin_fmaf(C, cy, Sn * sy);
    return S * ((sgn * (cw * cw)) * rx);
}

template <int M>
__device__ __forceinline__ void fwd_pair(int* __restrict__ row, float dl, float S, float cy, float sy,
                                         const float (&w)[kPowTerms], const float (&v)[kPowTerms]) {
    constexpr int J = kHalf + M, D = kPolyDeg[J];
    if constexpr (D < 0) {
        atomicAdd(row + kHalf + M, cvt_rpi_i32(tap_quotient<M>(dl, S, cy, sy)));
        atomicAdd(row + kHalf - M, cvt_rpi_i32(tap_quotient<-M>(dl, S, cy, sy)));
    } else {
        const float se = coef_chain<J, 0, 0, D / 2>(w);
        float so = 0.0f;
        if constexpr (D >= 1) so = coef_chain<J, 1, 0, (D - 1) / 2>(v);
        atomicAdd(row + kHalf + M, cvt_rpi_i32(se + so));
        atomicAdd(row + kHalf - M, cvt_rpi_i32(so - se));
    }
}

// All 81 taps of one pair: the centre (v0 = S Q_0, pre-scaled) and the
// mirrored pairs m = 1 .. 40.
template <int... M>
__device__ __forceinline__ void fwd_taps(std::integer_sequence<int, M...>, int* __restrict__ row, float dl, float S,
                                         float cy, float sy, float v0) {
    atomicAdd(row + kHalf, cvt_rpi_i32(v0));
    const float z = dl * dl;
    float w[kPowTerms], v[kPowTerms];
    w[0] = S;
    v[0] = S * dl;
#pragma unroll
    for (int j = 1; j < kPowTerms; ++j) {
        w[j] = w[j - 1] * z;
        v[j] = v[j - 1] * z;
    }
    (fwd_pair<M + 1>(row, dl, S, cy, sy, w, v), ...);
}

// ---- backward taps: s0 = sum_m G_m A P(m - dl), s1 = sum_m G_m A P'(m - dl)
// over the 81 taps of a pair (G_m: dL/dh at tap m).  With v = S Q_m(dl) and
// dS/ddl = A cos(pi dl) = Ac, A P'(m - dl) = -dv/ddl = -(Ac Q_m + S Q_m').
// For the polynomial taps the window folds into coefficient sums first,
//   sum_m G_m Q_m(dl) = sum_k dl^k D_k,   D_k = sum_m G_m c_{m,k},
// one FMA per coefficient, after which the sum and its derivative in dl are
// one Horner pass over D:
//   s0 += S p(dl),   s1 -= Ac p(dl) + S p'(dl),   p(dl) = sum_k D_k dl^k.
// The taps next to the centre use the closed form
//   A P'(x) = (1/x) [(-1)^m (A cos(pi dl) w + (2 pi/81) S sw cw) - A P(x)],
//   w = cw^2, cw = cos(pi x/81), sw = sin(pi x/81).
template <int J, int K>
__device__ __forceinline__ void fold_coef(float G, float (&D)[kPolyTop + 1]) {
    if constexpr (K <= kPolyDeg[J]) D[K] = __builtin_fmaf(G, kPolyCoef[J][K], D[K]);
}

template <int J, int... K>
__device__ __forceinline__ void fold_tap(float G, float (&D)[kPolyTop + 1], std::integer_sequence<int, K...>) {
    (fold_coef<J, K>(G, D), ...);
}

template <int J>
__device__ __forceinline__ void bwd_tap(const float* __restrict__ row, float (&D)[kPolyTop + 1], float cy, float sy,
                                        float dl, float S, float Ac, float S2, float v0, float dp0, float& s0,
                                        float& s1) {
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
        fold_tap<J>(G, D, std::make_integer_sequence<int, kPolyTop + 1>{});
    }
}

template <int... J>
__device__ __forceinline__ void bwd_taps(std::integer_sequence<int, J...>, const float* __restrict__ row, float cy,
                                         float sy, float dl, float S, float Ac, float S2, float v0, float dp0,
                                         float& s0, float& s1) {
    float D[kPolyTop + 1];
#pragma unroll
    for (int k = 0; k <= kPolyTop; ++k) D[k] = 0.0f;
    (bwd_tap<J>(row, D, cy, sy, dl, S, Ac, S2, v0, dp0, s0, s1), ...);
    float p = D[kPolyTop], dp = 0.0f;
#pragma unroll
    for (int k = kPolyTop - 1; k >= 0; --k) {
        dp = __builtin_fmaf(dp, dl, p);
        p = __builtin_fmaf(p, dl, D[k]);
    }
    s0 = __builtin_fmaf(S, p, s0);
    s1 = s1 - __builtin_fmaf(Ac, p, S * dp);
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
    double c0, hr, lm1, rl, rh;   // multi-rate plans: pulses on the high-rate grid (hr > 0)
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
    c.c0 = R->c;
    c.hr = R->hr;
    c.lm1 = R->lm1;
    c.rl = R->rl;
    c.rh = R->rh;
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

// ---------------------------------------------------------------------------
// Early-reverberation windows (Eq. 9) of a channel: its first output index,
// ceil(t0) - ceil(6 fs / 1000) with t0 = |src - mic| fs / c0 (correctly
// rounded square root, then one multiply and one divide, in this order).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t early_first(const RoomDesc* R, const double* p, const double* q) {
    const double dx = p[0] - q[0], dy = p[1] - q[1], dz = p[2] - q[2];
    const double t0 = (sqrt_rn(dx * dx + dy * dy + dz * dz) * R->fs) / R->c;
    return static_cast<int64_t>(__builtin_ceil(t0)) - R->early_pre;
}

// The render's share of the windows, for one item: the windows of its
// microphones take every output sample the item writes (early_put), and the
// item that starts a channel (t0 = 0) writes the window's start index and its
// samples before 0, the one that ends it (t0 + len >= T) those from T on.
// first: the group's window starts (int32: |start| < 2^31), in LDS.
struct EarlyItem {
    float* base;        // window of the group's first microphone (NULL: no windows requested)
    int width;
};

__device__ __forceinline__ void early_put(const EarlyItem& E, const int32_t* first, int mm, int64_t n, float v) {
    const int64_t j = n - first[mm];
    if (j >= 0 && j < E.width) E.base[static_cast<int64_t>(mm) * E.width + j] = v;
}

// The group's window starts into LDS (threads tid < mg; the caller
// synchronises), then zeros outside [0, T) and the start indices.
__device__ __forceinline__ EarlyItem early_item(const RoomDesc* R, float* __restrict__ early, int local0,
                                                const double* src_pos, const double* micq, int32_t* first, int mg,
                                                int tid) {
    EarlyItem E;
    E.width = R->early_pre + R->early_post + 1;
    E.base = early + R->early_off + static_cast<int64_t>(local0) * E.width;
    if (tid < mg) first[tid] = static_cast<int32_t>(early_first(R, src_pos, micq + 3 * tid));
    return E;
}

__device__ __forceinline__ void early_edges(const EarlyItem& E, const int32_t* first, const RoomDesc* R, int local0,
                                            int mg, int t0, int len, int32_t* __restrict__ start, int tid, int nt) {
    for (int mm = 0; mm < mg; ++mm) {
        float* e = E.base + static_cast<int64_t>(mm) * E.width;
        if (t0 == 0) {
            for (int64_t j = tid; j < E.width && first[mm] + j < 0; j += nt) e[j] = 0.0f;
            if (start && tid == 0) start[R->chan0 + local0 + mm] = static_cast<int32_t>(first[mm]);
        }
        if (t0 + len >= R->T)
            for (int64_t j = max(int64_t(0), R->T - first[mm]) + tid; j < E.width; j += nt) e[j] = 0.0f;
    }
}

// ---------------------------------------------------------------------------
// Render: fixed-point scale, preparation and the scatter kernel
// ---------------------------------------------------------------------------
// Fixed-point budget of the LDS accumulators.  A sample n of a source's RIR
// at any microphone only receives pulses of images whose centre delay lies
// within H = 43 + rho fs / c samples of n (half the pulse, plus the largest
// microphone offset from the array centre, plus rounding slack), and each
// adds at most r^g / D there, since the pulse never exceeds 1 in magnitude.
// The bound is therefore the largest sum of those terms over any window of
// delay bins an interval of 2H samples can touch (for a multi-rate room every
// window that reaches the clamped end runs to the last bin, since delays past
// the RIR length are clamped onto its last sample).  That bound plus the
// per-add rounding slack is mapped just below 2^31; the accumulators add
// modulo 2^32, so only each sample's final sum has to fit.
constexpr float kFixedBudget = 2147483648.0f - 262144.0f;
constexpr float kBoundMargin = 1.0001f;
constexpr int kBoundBins = 256;                     // bins of 4 delay buckets
constexpr int kBinShift = 2;
static_assert(kBuckets == (kBoundBins << kBinShift) && kBoundBins % 64 == 0, "delay bins");

// ---------------------------------------------------------------------------
// Render preparation: one workgroup per source.
//   - the fixed-point scale of the source: budget / the largest windowed sum
//     of max_m r^g_i / D_im, with D_im >= |pos_i - centre| - rho (rho =
//     largest |mic - centre| of the room), rows inside that sphere using the
//     exact nearest microphone; per-wave bin sums combined in a fixed order,
//     so the scale is reproducible;
//   - a counting sort of the source's rows by centre delay into kBuckets
//     buckets: bucket offsets, and the rows themselves stored in that order
//     as render rows (position, amplitude r^g as FP32).  A time tile then
//     reads one contiguous, coalesced range of rows.  Order inside a bucket
//     is arbitrary: the render accumulates integers, so its result does not
//     depend on it.
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

// A render row in 32 bytes: image position (FP64), then the amplitude r^g
// (FP32, low word) and the reflection count g (FP32, high word).
__device__ __forceinline__ double4 pack_render_row(const double4& v, float amp) {
    const unsigned long long lo = static_cast<unsigned>(__float_as_int(amp));
    const unsigned long long hi = static_cast<unsigned>(__float_as_int(static_cast<float>(v.w)));
    return make_double4(v.x, v.y, v.z, __longlong_as_double(static_cast<long long>(lo | (hi << 32))));
}

__device__ __forceinline__ float render_row_amp(double w) {
    return __int_as_float(static_cast<int>(static_cast<unsigned long long>(__double_as_longlong(w))));
}

__device__ __forceinline__ float render_row_g(double w) {
    return __int_as_float(static_cast<int>(static_cast<unsigned long long>(__double_as_longlong(w)) >> 32));
}

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

// Per-row accounting of the first pass: amplitude, the row's term of the
// amplitude bound, and its delay bucket.
__device__ __forceinline__ int prep_account(const RoomDesc* R, const double4& v, double log2r, float rhof,
                                            float inv_w, const double* __restrict__ mic, float& amp, float& term) {
    float dc;
    const float tc = prep_key_tc(R, v.x, v.y, v.z, dc);
    amp = exp2f(static_cast<float>(v.w * log2r));
    float dmin = dc * 0.999999f - rhof;
    if (dmin < 1e-3f) {
        dmin = 3.0e38f;
        for (int m = 0; m < R->n_mic; ++m) {
            const double* q = mic + 3 * (R->mic0 + m);
            const float dx = static_cast<float>(v.x - q[0]), dy = static_cast<float>(v.y - q[1]),
                        dz = static_cast<float>(v.z - q[2]);
            dmin = fminf(dmin, __builtin_sqrtf(__builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz))) * 0.999999f);
        }
    }
    term = amp / dmin;
    return bucket_of(tc, inv_w);
}

// The preparation runs kPrepThreads per source; each wave owns a contiguous
// range of the source's rows.  Dynamic LDS: bucket indices (u16) of the
// first key_cap rows.  kMaxImg: rows of a source at most (img_hi <= 65535,
// plus the direct path).
constexpr int kPrepThreads = 512;
constexpr int kPrepWaves = kPrepThreads / 64;
static_assert(kBoundBins <= kPrepThreads, "one thread per delay bin");
constexpr int kMaxImg = 65536;
__host__ __device__ constexpr int prep_key_cap(int max_img) { return ((max_img < kKeyCap ? max_img : kKeyCap) + 1) & ~1; }
__host__ __device__ constexpr int prep_dyn_lds(int max_img) { return 2 * prep_key_cap(max_img); }

template <bool DRAW>
__global__ void __launch_bounds__(kPrepThreads) prep_kernel(const void* __restrict__ desc, double* __restrict__ table,
                                                            const double* __restrict__ mic,
                                                            const double* __restrict__ src,
                                                            const double* __restrict__ r_in,
                                                            float* __restrict__ src_scale,
                                                            int* __restrict__ bucket_off, int* __restrict__ row0_slot,
                                                            int* __restrict__ room_done, double* __restrict__ sorted,
                                                            int key_cap) {
    constexpr int NT = kPrepThreads, NW = kPrepWaves, BPT = kBuckets / NT;
    extern __shared__ unsigned short keys[];             // key_cap
    __shared__ int hist[NW][kBuckets];                   // per-wave bucket counts, then per-wave cursors
    __shared__ float tsum[NW][kBoundBins];               // per-wave bound terms per delay bin
    __shared__ float bins[kBoundBins];
    __shared__ float red[NW];
    __shared__ int wsum[NW];
    __shared__ float s_rho;
    const DescHeader* H = hdr(desc);
    if (static_cast<int>(blockIdx.x) >= H->n_src) return;
    const int s = src_order(desc)[blockIdx.x];
    const SrcDesc* S = srcs(desc) + s;
    const RoomDesc* R = rooms(desc) + S->room;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int k = tid; k < NW * kBuckets; k += NT) (&hist[0][0])[k] = 0;
    for (int k = tid; k < NW * kBoundBins; k += NT) (&tsum[0][0])[k] = 0.0f;
    if (tid == 0) {
        s_rho = 0.0f;
        if (S->s_local == 0) room_done[S->room] = 0;   // completion count of the room's backward items
    }
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
    // rows read back from the table; none when drawing without one (the
    // second pass then draws each row again)
    const double4* trow = table ? reinterpret_cast<const double4*>(table) + S->img_off : nullptr;
    const double4 src_row = make_double4(src[3 * s], src[3 * s + 1], src[3 * s + 2], 0.0);
    // this wave's rows: [w0, w1), in runs of 64
    const int per_wave = (((n + NW - 1) / NW) + 63) & ~63;
    const int w0 = min(n, wave * per_wave), w1 = min(n, w0 + per_wave);
    __syncthreads();
    const float rhof = s_rho * 1.000001f + 1e-7f;
    // pass 1: rows (drawn and stored when DRAW), bound terms, buckets and the
    // wave's bucket counts and bin sums
    auto count_run = [&](int i, bool valid, const double4& v) {
        if (valid) {
            float amp, term;
            const int key = prep_account(R, v, log2r, rhof, inv_w, mic, amp, term);
            if (i < key_cap) keys[i] = static_cast<unsigned short>(key);
            atomicAdd(&hist[wave][key], 1);
            atomicAdd(&tsum[wave][key >> kBinShift], term);
        }
    };
    if constexpr (DRAW) {
        // two independent rows per lane and iteration: their FP64 chains overlap
#pragma unroll 1
        for (int c = w0; c < w1; c += 128) {
            const int i0 = c + lane, i1 = c + 64 + lane;
            const bool valid0 = i0 < w1, valid1 = i1 < w1;
            double4 v0 = make_double4(0.0, 0.0, 0.0, 0.0), v1 = v0;
            if (valid0) v0 = prep_row<true>(H, S, R, s, i0, table, src, table != nullptr);
            if (valid1) v1 = prep_row<true>(H, S, R, s, i1, table, src, table != nullptr);
            count_run(i0, valid0, v0);
            if (c + 64 < w1) count_run(i1, valid1, v1);
        }
    } else {
        for (int c = w0; c < w1; c += 4 * 64) {   // four loads in flight per lane
            double4 v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int i = c + 64 * k + lane;
                v[k] = make_double4(0.0, 0.0, 0.0, 0.0);
                if (i < w1) v[k] = i == 0 ? src_row : trow[i];
            }
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (c + 64 * k < w1) count_run(c + 64 * k + lane, c + 64 * k + lane < w1, v[k]);
        }
    }
    __syncthreads();
    if (tid < kBoundBins) {   // bin totals, waves in a fixed order
        float t = 0.0f;
        for (int w = 0; w < NW; ++w) t += tsum[w][tid];
        bins[tid] = t;
    }
    // bucket totals, exclusive scan (BPT buckets per thread), then each
    // wave's cursor: the bucket's start plus the earlier waves' counts
    int tot[BPT], run = 0;
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
        tot[j] = 0;
        for (int w = 0; w < NW; ++w) tot[j] += hist[w][tid * BPT + j];
        run += tot[j];
    }
    int incl = run;
    for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(incl, off);
        if (lane >= off) incl += v;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    if (tid < kBoundBins) {   // the largest window sum (bins now complete)
        const float H = 43.0f + rhof * static_cast<float>(R->fs_over_c) * 1.0001f;
        const float cw = (R->T + 256.0f) * (1.0f / kBoundBins);
        const int len = min(kBoundBins, static_cast<int>(__builtin_ceilf(2.0f * H / cw)) + 4);
        int end = min(kBoundBins, tid + len);
        if (R->hr > 0.0) {   // multi-rate: windows that reach the clamped end run to the last bin
            const int kc = (bucket_of(R->T - 2.0f * H - 4.0f, inv_w) >> kBinShift) - 1;
            if (tid >= kc) end = kBoundBins;
        }
        float wsum_bins = 0.0f;
        for (int k = tid; k < end; ++k) wsum_bins += bins[k];
        for (int off = 32; off > 0; off >>= 1) wsum_bins = fmaxf(wsum_bins, __shfl_xor(wsum_bins, off));
        if (lane == 0) red[wave] = wsum_bins;
    }
    int base = incl - run;
    for (int w = 0; w < wave; ++w) base += wsum[w];
    int* bo = bucket_off + static_cast<int64_t>(s) * (kBuckets + 1);
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
        const int b = tid * BPT + j;
        bo[b] = base;
        int cur = base;
        for (int w = 0; w < NW; ++w) {
            const int c = hist[w][b];
            hist[w][b] = cur;
            cur += c;
        }
        base += tot[j];
    }
    if (tid == 0) bo[kBuckets] = n;
    __syncthreads();
    if (tid == 0) {
        float b = 0.0f;
        for (int w = 0; w < kBoundBins / 64; ++w) b = fmaxf(b, red[w]);
        b *= kBoundMargin;
        src_scale[s] = (b > 0.0f && b < 3.0e38f) ? kFixedBudget / b : 0.0f;
    }
    // pass 2: each wave places its rows through its own cursors, runs of 64
    // in row order.  Only this wave touches its cursors, and one LDS atomic
    // instruction resolves its colliding lanes in a fixed order, so the
    // layout, and every sum later taken over it, is a function of the input
    // alone.  Rows come back from the table (for DRAW the lane's own stores
    // of pass 1), or are drawn again when there is no table.
    double4* dst = reinterpret_cast<double4*>(sorted) + S->img_off;
    for (int c = w0; c < w1; c += 4 * 64) {
        double4 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int i = c + 64 * k + lane;
            v[k] = make_double4(0.0, 0.0, 0.0, 0.0);
            if constexpr (DRAW) {
                if (i < w1) v[k] = trow ? (i == 0 ? src_row : trow[i]) : prep_row<true>(H, S, R, s, i, nullptr, src, false);
            } else {
                if (i < w1) v[k] = i == 0 ? src_row : trow[i];
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (c + 64 * k >= w1) continue;   // uniform per wave
            const int i = c + 64 * k + lane;
            const bool valid = i < w1;
            int key = 0;
            float amp = 0.0f;
            if (valid) {
                if (i < key_cap) {
                    key = keys[i];
                    amp = exp2f(static_cast<float>(v[k].w * log2r));
                } else {   // the same arithmetic on the same row gives the same bucket
                    float term;
                    key = prep_account(R, v[k], log2r, rhof, inv_w, mic, amp, term);
                }
            }
            if (valid) {
                const int slot = atomicAdd(&hist[wave][key], 1);
                dst[slot] = pack_render_row(v[k], amp);
                if (i == 0) row0_slot[s] = slot;   // where the direct path landed
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Render
// ---------------------------------------------------------------------------
// LDS bank-aware scheduling of the scatter.  gfx950's LDS has 32 banks of 4
// bytes and serves an atomic instruction one half-wave (32 lanes) at a time;
// a half-wave costs max(2, largest number of its lanes in one bank) cycles.
// The lanes of one tap instruction address word (first tap + j) of their
// pairs, so their banks are those of the first taps, shifted alike: pairs
// whose first taps share a bank collide on all 81 taps.  A pool of 128 pairs
// sorted by that bank and dealt round-robin to four half-waves puts at most
// ceil(c / 4) pairs of a bank into one half-wave, c being the pool's pairs in
// that bank (about Poisson(4)), against about Poisson(1) per bank for 32
// lanes that take pairs as they come.  Integer sums do not depend on the
// order, so neither does the output.

// What a tap phase needs of a pair: the LDS word of its first tap, dl and
// (A x fixed-point scale) sinc(dl); cos, sin of pi dl / 81 and S are
// recomputed from dl.
struct StagedPair {
    int word;      // LDS word of tap 0, or -1 when the pair adds nothing to this tile
    float dl;
    float as;
};

template <typename Ctx>
__device__ __forceinline__ StagedPair stage_pair(const Ctx& c, const double4& row, const double* q, int row_base,
                                                 int shift, float scale, bool live) {
    StagedPair sp{-1, 0.0f, 0.0f};
    if (!live) return sp;
    const Pair P = c.hr > 0.0 ? pair_setup_high_rate(row.x, row.y, row.z, q[0], q[1], q[2], c.c0, c.hr, c.lm1,
                                                     c.rl, c.rh, render_row_amp(row.w))
                              : pair_setup(row.x, row.y, row.z, q[0], q[1], q[2], c.fs_over_c, render_row_amp(row.w));
    const int b0 = P.k + shift;   // tap 0 within the microphone's row
    if (b0 < 0 || b0 + kTaps > c.rowlen) return sp;
    sp.word = row_base + b0;
    sp.dl = P.dl;
    sp.as = (P.A * scale) * P.sinc;
    return sp;
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One round of a wave: rank the pool by bank, stage it in dealt order, run
// the taps of two wave-steps (four half-waves).
__device__ __forceinline__ void pool_round(int* __restrict__ acc, uint32_t* __restrict__ st, int* __restrict__ cnt,
                                           int lane, const StagedPair& a, const StagedPair& b) {
    if (lane < kLdsBanks) cnt[lane] = 0;
    wave_sync();
    const int ka = a.word & (kLdsBanks - 1), kb = b.word & (kLdsBanks - 1);
    int ra = 0, rb = 0;
    if (a.word >= 0) ra = atomicAdd(&cnt[ka], 1);
    if (b.word >= 0) rb = atomicAdd(&cnt[kb], 1);
    wave_sync();
    // exclusive scan of the bank counts (lanes 0..31) in registers (DPP row
    // shifts, then lane 15 broadcast into the next row), not through the LDS
    // queue that the tap atomics keep busy
    const int cv = lane < kLdsBanks ? cnt[lane] : 0;
    int incl = cv;
    incl += __builtin_amdgcn_update_dpp(0, incl, 0x111, 0xf, 0xf, false);   // row_shr:1
    incl += __builtin_amdgcn_update_dpp(0, incl, 0x112, 0xf, 0xf, false);   // row_shr:2
    incl += __builtin_amdgcn_update_dpp(0, incl, 0x114, 0xf, 0xf, false);   // row_shr:4
    incl += __builtin_amdgcn_update_dpp(0, incl, 0x118, 0xf, 0xf, false);   // row_shr:8
    incl += __builtin_amdgcn_update_dpp(0, incl, 0x142, 0xa, 0xf, false);   // row_bcast:15 into rows 1, 3
    const int n_pool = __builtin_amdgcn_readlane(incl, kLdsBanks - 1);
    wave_sync();
    if (lane < kLdsBanks) cnt[lane] = incl - cv;
    wave_sync();
    // position pi in bank order -> half-wave pi mod H, slot pi / H, with H
    // = ceil(n_pool / 32) half-waves (a partly filled pool runs fewer)
    const int H = (n_pool + 31) >> 5;
    const int hmul = H == 3 ? 21846 : 65536 / max(H, 1);    // pi / H = (pi hmul) >> 16 for pi < 128
    if (a.word >= 0) {
        const int pi = cnt[ka] + ra, i = (pi * hmul) >> 16, q = (pi - i * H) * 32 + i;
        st[q] = static_cast<uint32_t>(a.word);
        st[kPool + q] = __float_as_uint(a.dl);
        st[2 * kPool + q] = __float_as_uint(a.as);
    }
    if (b.word >= 0) {
        const int pi = cnt[kb] + rb, i = (pi * hmul) >> 16, q = (pi - i * H) * 32 + i;
        st[q] = static_cast<uint32_t>(b.word);
        st[kPool + q] = __float_as_uint(b.dl);
        st[2 * kPool + q] = __float_as_uint(b.as);
    }
    wave_sync();
#pragma unroll 1
    for (int step = 0; 2 * step < H; ++step) {
        const int q = 64 * step + lane;                        // half-wave h = q / 32, slot i = q % 32
        const int h = q >> 5;
        if (h < H && (lane & 31) * H + h < n_pool) {
            const int word = static_cast<int>(st[q]);
            const float dl = __uint_as_float(st[kPool + q]);
            const float as = __uint_as_float(st[2 * kPool + q]);
            const float y = (kPiF / 81.0f) * dl;
            const float y2 = y * y;
            // |y| <= pi / 162: three Taylor terms are exact to FP32 rounding
            const float cy = __builtin_fmaf(y2, __builtin_fmaf(y2, 1.0f / 24.0f, -0.5f), 1.0f);
            const float sy = y * __builtin_fmaf(y2, __builtin_fmaf(y2, 1.0f / 120.0f, -1.0f / 6.0f), 1.0f);
            fwd_taps(std::make_integer_sequence<int, kHalf>{}, acc + word, dl, as * dl, cy, sy, as * (cy * cy));
        }
    }
    wave_sync();
}

template <int NT, int WPE, bool EARLY>   // EARLY: the Eq. 9 windows are written too
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE)))
render_kernel(const void* __restrict__ desc, const double* __restrict__ table, const double* __restrict__ mic,
              const double* __restrict__ src, const double* __restrict__ r_in, float* __restrict__ out,
              int* __restrict__ counters, const float* __restrict__ src_scale, const int* __restrict__ bucket_off,
              const double* __restrict__ sorted, int acc_words, float* __restrict__ early,
              int32_t* __restrict__ early_start) {
    extern __shared__ int acc[];
    __shared__ double micq[3 * kMaxMicGroup];
    __shared__ int32_t s_efirst[kMaxMicGroup];        // early windows: starts of the group's channels
    __shared__ int s_item;
    __shared__ uint32_t stage[NT / 64][3 * kPool];   // per wave: staged pairs of a round
    __shared__ int bank_cnt[NT / 64][kLdsBanks];
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
        const double4* rows = reinterpret_cast<const double4*>(sorted) + c.img_off + lo;
        const int n_list = hi - lo;
        // The range is in delay order; visiting it as j = e * P mod n_list
        // (P prime, coprime to n_list) hands the lanes of a wave rows spread
        // over the whole range, so their LDS adds rarely meet in one word.
        int P = 97;                          // 97, 89, 83: their product exceeds any row count
        while (n_list > 0 && n_list % P == 0) P = (P == 97) ? 89 : 83;
        const int jstep = n_list > 0 ? static_cast<int>((static_cast<int64_t>(NT) * P) % n_list) : 0;
        __syncthreads();
        // ---- scatter the taps as rounded fixed-point integers.  Pair
        // p = m * n_list + e: a wave takes rows of one microphone.  Each
        // round a wave sets up two pairs per lane (p and p + NT), ranks its
        // pool of up to 128 by the LDS bank of the pair's first tap and
        // deals that order round-robin into four half-waves, then runs the
        // taps from the staged pairs (pool_round).
        const int n_pairs = n_list * mg;
        const int lane = tid & 63;
        int m = 0, e = tid;                 // (m, e) of the lane's next pair, advanced without division
        while (e >= n_list && m < mg) {
            e -= n_list;
            ++m;
        }
        int j = n_list > 0 ? static_cast<int>((static_cast<int64_t>(e) * P) % n_list) : 0;
        auto advance = [&]() {
            e += NT;
            j += jstep;
            if (j >= n_list) j -= n_list;
            while (e >= n_list && m < mg) {
                e -= n_list;
                ++m;
            }
        };
        double4 rowA = make_double4(0.0, 0.0, 0.0, 0.0), rowB = rowA;
        int mA = m;
        if (tid < n_pairs) rowA = rows[j];
        advance();
        int mB = m;
        if (tid + NT < n_pairs) rowB = rows[j];
        advance();
        for (int p0 = tid - lane; p0 < n_pairs; p0 += 2 * NT) {   // wave-uniform: p0 is lane 0's pair
            const int pA = p0 + lane, pB = pA + NT;
            const StagedPair a = stage_pair(c, rowA, micq + 3 * mA, mA * c.rowlen, shift, scale, pA < n_pairs);
            const StagedPair b = stage_pair(c, rowB, micq + 3 * mB, mB * c.rowlen, shift, scale, pB < n_pairs);
            // the next round's rows load while this round's taps run
            mA = m;
            if (pA + 2 * NT < n_pairs) rowA = rows[j];
            advance();
            mB = m;
            if (pB + 2 * NT < n_pairs) rowB = rows[j];
            advance();
            pool_round(acc, stage[tid >> 6], bank_cnt[tid >> 6], lane, a, b);
        }
        __syncthreads();
        // writeback of the tile core, samples [t0, min(t0 + len, T)), and
        // clearing of every accumulator the item touched
        const int nvalid = min(c.w.len, c.T - c.w.t0);
        const float inv = scale > 0.0f ? 1.0f / scale : 0.0f;
        const int local0 = c.s_local * c.n_mic_room + c.w.mic0;   // the group's first channel in the room
        EarlyItem E{nullptr, 0};
        if constexpr (EARLY) {
            const RoomDesc* R = rooms(desc) + c.room;
            E = early_item(R, early, local0, src + 3 * c.w.src, micq, s_efirst, mg, tid);
            __syncthreads();
            early_edges(E, s_efirst, R, local0, mg, c.w.t0, c.w.len, early_start, tid, NT);
        }
        for (int mm = 0; mm < mg; ++mm) {
            float* dst = out + c.out_off + static_cast<int64_t>(local0 + mm) * c.T + c.w.t0;
            int* row = acc + mm * c.rowlen;
            for (int k = tid; k < c.rowlen; k += NT) {
                const int v = row[k];
                if (k >= kHalo && k < kHalo + nvalid) {
                    const float h = static_cast<float>(v) * inv;
                    dst[k - kHalo] = h;
                    if constexpr (EARLY) early_put(E, s_efirst, mm, c.w.t0 + k - kHalo, h);
                }
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
// Render by bin moments (the second render path)
// ---------------------------------------------------------------------------
// For the taps |m| >= 3 the pulse is a polynomial in the fractional delay of
// degree <= 5 (tap_poly.h): A P(m - dl) = S Q_m(dl) = sum_k c_{m,k} 2^-k
// S (2 dl)^k.  Summed over the pairs whose centre tap falls on sample K (k =
// K), sample n of a channel receives
//   h[n] = sum_{|m| >= 3} sum_k (c_{m,k} 2^-k) U_k[n - m] + centre taps,
//   U_k[K] = sum over those pairs of S (2 dl)^k,
// so a pair adds its six moments U_0..U_5 to its bin and its five centre taps
// (m = 0, +-1, +-2, quotient form) to a direct row: 11 LDS atomics instead of
// 81.  The moments are fixed-point integers under the source's scale
// ((2 dl)^k <= 1 keeps each inside the budget), added with ds_add_u32, so
// their sums do not depend on the order of the additions.
// The sum over m is a fixed banded (Toeplitz) product per power k, done on
// the matrix cores: a block of 256 output samples of one microphone is a
// 16 x 16 tile D[i][b] = h[n0 + 16 b + i] = sum_k W_k X_k, with W_k[i][q] =
// c_{i-q+40,k} 2^-k (zero outside the band and for |m| < 3) and X_k[q][b] =
// U_k[n0 + 16 b - 40 + q], q in [0, 96).  Operands are fp16: a moment enters
// as v = U 2^-16 split into hi = fp16(v) and lo = fp16(v - hi), a coefficient
// likewise, and the FP32 accumulator takes hi*hi + hi*lo + lo*hi (powers 0-2;
// for powers 3-5, whose terms are at most 2^-9 of the sum, hi*hi), so every
// term keeps about 22 bits.  Integer bins and a fixed MFMA order make the
// output bitwise reproducible.

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

constexpr int kMomPow = 6;        // moments U_0 .. U_5
constexpr int kMomSplit = 3;      // powers below this use hi + lo operands
constexpr int kMomSteps = 13;     // K-steps of 32 over (power, q)
constexpr int kMomStepPow[kMomSteps] = {0, 0, 0, 1, 1, 1, 2, 2, 2, 3, 3, 4, 5};
constexpr int kMomStepQ[kMomSteps] = {0, 32, 64, 0, 32, 64, 0, 32, 64, 16, 48, 32, 32};
constexpr float kMomSigma = 1.0f / 65536.0f;   // |U| < 2^31, so |U 2^-16| < 2^15 fits fp16
constexpr int kMomGroup = 4;     // 256-sample blocks a wave runs side by side

constexpr float pow2i(int e) {
    float v = 1.0f;
    for (; e > 0; --e) v *= 2.0f;
    for (; e < 0; ++e) v *= 0.5f;
    return v;
}

// Every nonzero W_k[i][q] lies in exactly one K-step of its power, every
// polynomial tap has degree < kMomPow, and the steps stay inside q < 96.
constexpr bool mom_steps_cover() {
    for (int m = 3; m <= kHalf; ++m)
        if (kPolyDeg[kHalf + m] >= kMomPow || kPolyDeg[kHalf - m] >= kMomPow) return false;
    for (int s = 0; s < kMomSteps; ++s) {
        if (kMomStepQ[s] < 0 || kMomStepQ[s] + 32 > 2 * kHalf + 16) return false;
        for (int t = s + 1; t < kMomSteps; ++t)
            if (kMomStepPow[s] == kMomStepPow[t] && kMomStepQ[s] < kMomStepQ[t] + 32 &&
                kMomStepQ[t] < kMomStepQ[s] + 32)
                return false;
    }
    for (int k = 0; k < kMomPow; ++k)
        for (int m = -kHalf; m <= kHalf; ++m) {
            if ((m > -3 && m < 3) || k > kPolyDeg[kHalf + m]) continue;
            for (int i = 0; i < 16; ++i) {
                const int q = i - m + kHalf;
                bool hit = false;
                for (int s = 0; s < kMomSteps; ++s)
                    if (kMomStepPow[s] == k && q >= kMomStepQ[s] && q < kMomStepQ[s] + 32) hit = true;
                if (!hit) return false;
            }
        }
    return true;
}
static_assert(mom_steps_cover(), "the K-steps must cover the band of every power exactly once");

constexpr uint32_t f16_bits(float x) { return __builtin_bit_cast(uint16_t, static_cast<_Float16>(x)); }

// W_k fragments in the MFMA A-operand layout of v_mfma_f32_16x16x32_f16
// (lane l: row l % 16, columns 8 (l / 16) .. + 7 of the step), hi and lo.
struct alignas(16) MomFrags {
    uint32_t w[kMomSteps][2][64][4];
    constexpr MomFrags() : w{} {
        for (int s = 0; s < kMomSteps; ++s)
            for (int l = 0; l < 64; ++l)
                for (int e = 0; e < 8; ++e) {
                    const int k = kMomStepPow[s];
                    const int i = l % 16, q = kMomStepQ[s] + 8 * (l / 16) + e, m = i - q + kHalf;
                    float c = 0.0f;
                    if (m >= -kHalf && m <= kHalf && (m <= -3 || m >= 3) && k <= kPolyDeg[kHalf + m])
                        c = kPolyCoef[kHalf + m][k] * pow2i(-k);
                    const float hi = static_cast<float>(static_cast<_Float16>(c));
                    const float lo = k < kMomSplit ? c - hi : 0.0f;
                    w[s][0][l][e / 2] |= f16_bits(hi) << (16 * (e & 1));
                    w[s][1][l][e / 2] |= f16_bits(lo) << (16 * (e & 1));
                }
    }
};
__device__ constexpr MomFrags kMomFrags{};

__device__ __forceinline__ f32x4 mfma_16x16x32(const u32x4& a, const u32x4& b, const f32x4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0,
                                                  0, 0);
}

// In-place conversion of the moment rows of an item to fp16 operands, each
// thread rewriting only the words it reads (no barrier inside):
//   rows 0 .. kMomSplit-1, bins (2p, 2p+1) in words (2p, 2p+1) become
//     word 2p = hi halves of both bins, word 2p+1 = lo halves;
//   the other rows, bins 4p .. 4p+3 in words 4p .. 4p+3 become
//     words 4p, 4p+1 = hi halves of the four bins (4p+2, 4p+3 unused).
// Bin e's hi half thus sits in word e & ~1 (split rows) or (e & ~3) + (e & 3)/2
// (hi-only rows), low or high half by e & 1.
__device__ __forceinline__ uint32_t pack_f16(float a, float b) {
    return static_cast<uint32_t>(__builtin_bit_cast(uint16_t, static_cast<_Float16>(a))) |
           (static_cast<uint32_t>(__builtin_bit_cast(uint16_t, static_cast<_Float16>(b))) << 16);
}

__device__ __forceinline__ float f16_lo_of(uint32_t w) {
    return static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(w & 0xffffu)));
}

__device__ __forceinline__ float f16_hi_of(uint32_t w) {
    return static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(w >> 16)));
}

__device__ __forceinline__ int mom_word(int e) { return e + 4 * (e >> 5); }

template <int NT>
__device__ __forceinline__ void mom_convert(int* __restrict__ lds, int mg, int Rw, int tid) {
    // the rows are converted whole, pad words included (they hold zeros)
    for (int m = 0; m < mg; ++m) {
        int* base = lds + m * (kMomRows * Rw);
        // split rows: kMomSplit Rw words as pairs
        int2* sp = reinterpret_cast<int2*>(base);
        for (int p = tid; p < (kMomSplit * Rw) / 2; p += NT) {
            const int2 u = sp[p];
            const float a = static_cast<float>(u.x) * kMomSigma, b = static_cast<float>(u.y) * kMomSigma;
            const uint32_t hw = pack_f16(a, b);
            const uint32_t lw = pack_f16(a - f16_lo_of(hw), b - f16_hi_of(hw));
            sp[p] = make_int2(static_cast<int>(hw), static_cast<int>(lw));
        }
        // hi-only rows: (kMomPow - kMomSplit) Rw words as quads
        i32x4* qp = reinterpret_cast<i32x4*>(base + kMomSplit * Rw);
        for (int p = tid; p < ((kMomPow - kMomSplit) * Rw) / 4; p += NT) {
            const i32x4 u = qp[p];
            const uint32_t h0 = pack_f16(static_cast<float>(u[0]) * kMomSigma, static_cast<float>(u[1]) * kMomSigma);
            const uint32_t h1 = pack_f16(static_cast<float>(u[2]) * kMomSigma, static_cast<float>(u[3]) * kMomSigma);
            *reinterpret_cast<int2*>(qp + p) = make_int2(static_cast<int>(h0), static_cast<int>(h1));
        }
    }
}

// The rows of an item's tile and a thread's walk over its pairs (p = m
// n_list + e, row j = e P mod n_list with P prime, coprime to n_list, so that
// the lanes of a wave take rows spread over the delay range); the first row
// is loaded on set-up, so that it can be issued an item ahead.
struct MomWalk {
    const double4* rows;
    int n_list, n_pairs, jstep, m, e, j, p;
    double4 row;
};

template <int NT>
__device__ __forceinline__ void mom_walk_init(MomWalk& w, const ItemCtx& c, const int* __restrict__ bucket_off,
                                              const double* __restrict__ sorted, int tid) {
    int lo = 0, hi = c.n_img;
    if (!c.w.full) {
        const float inv_w = bucket_inv_width(c.T);
        const int b_lo = bucket_of(c.w.t0 - c.margin - 41.0f, inv_w);
        const int b_hi = bucket_of((c.w.t0 + c.w.len + c.margin + 41.0f), inv_w);
        const int* bo = bucket_off + static_cast<int64_t>(c.w.src) * (kBuckets + 1);
        lo = bo[b_lo];
        hi = bo[b_hi + 1];
    }
    w.rows = reinterpret_cast<const double4*>(sorted) + c.img_off + lo;
    w.n_list = hi - lo;
    int P = 97;
    while (w.n_list > 0 && w.n_list % P == 0) P = (P == 97) ? 89 : 83;
    w.jstep = w.n_list > 0 ? static_cast<int>((static_cast<int64_t>(NT) * P) % w.n_list) : 0;
    w.n_pairs = w.n_list * c.w.n_mic;
    w.m = 0;
    w.e = tid;
    while (w.e >= w.n_list && w.m < c.w.n_mic) {
        w.e -= w.n_list;
        ++w.m;
    }
    w.j = w.n_list > 0 ? static_cast<int>((static_cast<int64_t>(w.e) * P) % w.n_list) : 0;
    w.p = tid;
    w.row = make_double4(0.0, 0.0, 0.0, 0.0);
    if (tid < w.n_pairs) w.row = w.rows[w.j];
}

template <int NT, int WPE, bool EARLY>   // EARLY: the Eq. 9 windows are written too
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE)))
render_moment_kernel(const void* __restrict__ desc, const double* __restrict__ mic, const double* __restrict__ src,
                     const double* __restrict__ r_in, float* __restrict__ out, int* __restrict__ counters,
                     const float* __restrict__ src_scale, const int* __restrict__ bucket_off,
                     const double* __restrict__ sorted, int lds_words, float* __restrict__ early,
                     int32_t* __restrict__ early_start) {
    extern __shared__ u32x4 lds_v[];
    int* lds = reinterpret_cast<int*>(lds_v);
    __shared__ double micq[3 * kMaxMicGroup];
    __shared__ int32_t s_efirst[kMaxMicGroup];        // early windows: starts of the group's channels
    __shared__ int s_item;
    const DescHeader* H = hdr(desc);
    const int n_items = H->n_items;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int NW = NT / 64;
    // bins start at zero; each item clears what it used
    for (int k = tid; k < (lds_words >> 2); k += NT) lds_v[k] = u32x4{0u, 0u, 0u, 0u};
    if (tid == 0) s_item = atomicAdd(&counters[0], 1);
    __syncthreads();
    int item = __builtin_amdgcn_readfirstlane(s_item);
    // The items run as a pipeline: the next item's queue slot is taken while
    // this one's bins are converted, and its descriptor, microphone positions
    // and first rows load while this one's filter runs on the matrix cores.
    ItemCtx c;
    MomWalk wk;
    if (item < n_items) {
        load_item(desc, item, mic, r_in, c);
        if (tid < 3 * c.w.n_mic) micq[tid] = mic[3 * c.mic0_glob + tid];
        mom_walk_init<NT>(wk, c, bucket_off, sorted, tid);
    }
    __syncthreads();
    while (item < n_items) {
        const int mg = c.w.n_mic;
        const int nblk = (c.w.len + kMomBlock - 1) / kMomBlock;
        const int R = nblk * kMomBlock + 2 * kHalf;   // bins t0 - 40 .. t0 + 256 nblk + 39
        const int Rw = mom_row_words(R);              // words of a row, pads included
        const int mic_words = kMomRows * Rw;
        const float scale = src_scale[c.w.src];
        // ---- scatter: per pair (row, microphone) six moments and five centre taps
        for (; wk.p < wk.n_pairs; wk.p += NT) {
            const double4 cur = wk.row;
            const int mc = wk.m;
            wk.e += NT;
            wk.j += wk.jstep;
            if (wk.j >= wk.n_list) wk.j -= wk.n_list;
            while (wk.e >= wk.n_list && wk.m < mg) {
                wk.e -= wk.n_list;
                ++wk.m;
            }
            if (wk.p + NT < wk.n_pairs) wk.row = wk.rows[wk.j];   // the next pair's row loads during this one
            const double* q = micq + 3 * mc;
            const Pair Pp = c.hr > 0.0 ? pair_setup_high_rate(cur.x, cur.y, cur.z, q[0], q[1], q[2], c.c0, c.hr,
                                                              c.lm1, c.rl, c.rh, render_row_amp(cur.w))
                                       : pair_setup(cur.x, cur.y, cur.z, q[0], q[1], q[2], c.fs_over_c,
                                                    render_row_amp(cur.w));
            const int bin = Pp.k - c.w.t0 + kHalf;
            if (bin < 0 || bin >= R) continue;
            int* base = lds + mc * mic_words;
            const float as = (Pp.A * scale) * Pp.sinc;   // A scale sinc(dl)
            const float S = as * Pp.dl;                    // A scale sin(pi dl) / pi
            const float x2 = Pp.dl + Pp.dl;
            const int wb = mom_word(bin);
            float mk = S;
#pragma unroll
            for (int k = 0; k < kMomPow; ++k) {
                atomicAdd(base + k * Rw + wb, cvt_rpi_i32(mk));
                mk *= x2;
            }
            int* dr = base + kMomPow * Rw;
            atomicAdd(dr + wb, cvt_rpi_i32(as * (Pp.cy * Pp.cy)));
            if (bin >= 1) atomicAdd(dr + mom_word(bin - 1), cvt_rpi_i32(tap_quotient<-1>(Pp.dl, S, Pp.cy, Pp.sy)));
            if (bin >= 2) atomicAdd(dr + mom_word(bin - 2), cvt_rpi_i32(tap_quotient<-2>(Pp.dl, S, Pp.cy, Pp.sy)));
            if (bin + 1 < R) atomicAdd(dr + mom_word(bin + 1), cvt_rpi_i32(tap_quotient<1>(Pp.dl, S, Pp.cy, Pp.sy)));
            if (bin + 2 < R) atomicAdd(dr + mom_word(bin + 2), cvt_rpi_i32(tap_quotient<2>(Pp.dl, S, Pp.cy, Pp.sy)));
        }
        __syncthreads();
        // ---- the next item's slot; moments to fp16 operands (in place)
        if (tid == 0) s_item = atomicAdd(&counters[0], 1);
        mom_convert<NT>(lds, mg, Rw, tid);
        __syncthreads();
        const int next = __builtin_amdgcn_readfirstlane(s_item);
        ItemCtx cn;
        MomWalk wn;
        if (next < n_items) {   // its loads are in flight during the filter
            load_item(desc, next, mic, r_in, cn);
            mom_walk_init<NT>(wn, cn, bucket_off, sorted, tid);
        }
        // ---- FIR on the matrix cores: a wave takes kMomGroup blocks of 256
        // samples side by side (independent accumulators); the coefficient
        // fragments come through a three-deep register ring, two steps ahead
        const float inv = scale > 0.0f ? 1.0f / scale : 0.0f;
        const float inv_mom = inv * (1.0f / kMomSigma);
        const int col = lane & 15, grp = lane >> 4;
        const int end = min(c.w.t0 + c.w.len, c.T);
        const int nb = mg * nblk;
        const int local0 = c.s_local * c.n_mic_room + c.w.mic0;   // the group's first channel in the room
        EarlyItem E{nullptr, 0};
        if constexpr (EARLY) {   // (micq still holds this item's microphones)
            const RoomDesc* Rr = rooms(desc) + c.room;
            E = early_item(Rr, early, local0, src + 3 * c.w.src, micq, s_efirst, mg, tid);
            __syncthreads();
            early_edges(E, s_efirst, Rr, local0, mg, c.w.t0, c.w.len, early_start, tid, NT);
        }
        for (int g0 = wave; g0 < nb; g0 += NW * kMomGroup) {
            f32x4 acc[kMomGroup];
            int eo0[kMomGroup], mo0[kMomGroup];
#pragma unroll
            for (int i = 0; i < kMomGroup; ++i) {
                acc[i] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
                const int blk = g0 + NW * i, mm = blk / nblk, beta = blk - mm * nblk;
                // bin of the lane's first operand at q = 0, and its microphone's rows
                eo0[i] = beta * kMomBlock + 16 * col + 8 * grp;
                mo0[i] = mm * mic_words;
            }
            // the lane index made opaque, so that the fragment loads stay in
            // the loop (registers) instead of being hoisted for the whole item
            int fl = lane;
            asm volatile("" : "+v"(fl));
            u32x4 fh[3], fo[3];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                fh[s] = *reinterpret_cast<const u32x4*>(kMomFrags.w[s][0][fl]);
                fo[s] = *reinterpret_cast<const u32x4*>(kMomFrags.w[s][1][fl]);
            }
#pragma unroll
            for (int s = 0; s < kMomSteps; ++s) {
                const int k = kMomStepPow[s];
                if (s + 2 < kMomSteps) {
                    fh[(s + 2) % 3] = *reinterpret_cast<const u32x4*>(kMomFrags.w[s + 2][0][fl]);
                    if (kMomStepPow[s + 2] < kMomSplit)
                        fo[(s + 2) % 3] = *reinterpret_cast<const u32x4*>(kMomFrags.w[s + 2][1][fl]);
                }
                const u32x4 ah = fh[s % 3], al = fo[s % 3];
#pragma unroll
                for (int i = 0; i < kMomGroup; ++i) {
                    if (g0 + NW * i >= nb) break;   // wave-uniform
                    // the 8 bins e .. e + 7 of the operand (e a multiple of 8:
                    // consecutive words inside one 32-bin run)
                    const int* w = lds + mo0[i] + k * Rw + mom_word(eo0[i] + kMomStepQ[s]);
                    if (k < kMomSplit) {
                        const u32x4 w0 = *reinterpret_cast<const u32x4*>(w);
                        const u32x4 w1 = *reinterpret_cast<const u32x4*>(w + 4);
                        const u32x4 bh = u32x4{w0[0], w0[2], w1[0], w1[2]};
                        const u32x4 bl = u32x4{w0[1], w0[3], w1[1], w1[3]};
                        acc[i] = mfma_16x16x32(ah, bh, acc[i]);
                        acc[i] = mfma_16x16x32(ah, bl, acc[i]);
                        acc[i] = mfma_16x16x32(al, bh, acc[i]);
                    } else {
                        const uint2 w0 = *reinterpret_cast<const uint2*>(w);
                        const uint2 w1 = *reinterpret_cast<const uint2*>(w + 4);
                        acc[i] = mfma_16x16x32(ah, u32x4{w0.x, w0.y, w1.x, w1.y}, acc[i]);
                    }
                }
                // one step's operands in flight at a time (bounds the registers)
                __builtin_amdgcn_sched_barrier(0);
            }
            // lane: samples n .. n + 3 (rows 4 grp .. 4 grp + 3 of column col)
#pragma unroll
            for (int i = 0; i < kMomGroup; ++i) {
                const int blk = g0 + NW * i;
                if (blk >= nb) break;
                const int mm = blk / nblk, beta = blk - mm * nblk;
                const int off = beta * kMomBlock + 16 * col + 4 * grp;
                const int n = c.w.t0 + off;
                const i32x4 d =
                    *reinterpret_cast<const i32x4*>(lds + mm * mic_words + kMomPow * Rw + mom_word(off + kHalf));
                float* dst = out + c.out_off + static_cast<int64_t>(local0 + mm) * c.T;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (n + r < end) {
                        const float h = __builtin_fmaf(acc[i][r], inv_mom, static_cast<float>(d[r]) * inv);
                        dst[n + r] = h;
                        if constexpr (EARLY) early_put(E, s_efirst, mm, n + r, h);
                    }
            }
        }
        __syncthreads();
        // clear this item's rows; the next item's microphones
        for (int k = tid; k < (mg * mic_words) >> 2; k += NT) lds_v[k] = u32x4{0u, 0u, 0u, 0u};
        if (next < n_items && tid < 3 * cn.w.n_mic) micq[tid] = mic[3 * cn.mic0_glob + tid];
        __syncthreads();
        item = next;
        c = cn;
        wk = wn;
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
// Sums the partials of room b's items in the plan's fixed order (room_items)
// into its gradient outputs.  scratch: at least 4 ints of LDS, staging the
// item table in chunks so that the partial loads do not chain.  DRAWS adds
// the terms through the draws (Eq. 4-6): with u0_s = (src_s - centre) / d0_s
// and dL/dd0_s the sum of the items' dL/dd0 partials,
//   dL/dsrc_s += dL/dd0_s u0_s,
//   dL/dmic_m += sum over the room's items of (sum dL/dpos - dL/dd0 u0_s) / M,
// the centre being the mean of the M microphones.
template <int NT, bool DRAWS>
__device__ void finalize_room(const void* __restrict__ desc, int b, const float* __restrict__ partials,
                              float* __restrict__ grad_mic, float* __restrict__ grad_src, float* __restrict__ grad_r,
                              int* __restrict__ scratch, int scratch_words) {
    const RoomDesc* R = rooms(desc) + b;
    const int32_t* ri = room_items(desc) + R->item0;
    const WorkItem* it = items(desc);
    const int n_mic3 = 3 * R->n_mic, n_src3 = 3 * R->n_src;
    const int n_out = n_mic3 + n_src3 + 1;
    const int chunk = scratch_words / 4;
    for (int ob = 0; ob < n_out; ob += NT) {
        const int o = ob + static_cast<int>(threadIdx.x);
        const int axis = o % 3;
        float sum = 0.0f, extra = 0.0f;   // extra: the centre term (microphones) or dL/dd0 (sources)
        for (int j0 = 0; j0 < R->n_item; j0 += chunk) {
            const int nj = min(chunk, R->n_item - j0);
            __syncthreads();
            for (int j = threadIdx.x; j < nj; j += NT) {
                const int id = ri[j0 + j];
                const WorkItem& w = it[id];
                scratch[4 * j] = id;
                scratch[4 * j + 1] = w.mic0;
                scratch[4 * j + 2] = w.n_mic;
                scratch[4 * j + 3] = w.src - R->src0;
            }
            __syncthreads();
            if (o < n_out) {
                for (int j = 0; j < nj; ++j) {
                    const int id = scratch[4 * j], mic0 = scratch[4 * j + 1], nm = scratch[4 * j + 2],
                              sl = scratch[4 * j + 3];
                    const float* part = partials + static_cast<int64_t>(id) * kPartialStride;
                    int at;   // this item's partial feeding output o, or -1
                    if (o < n_mic3) {
                        const int m = o / 3 - mic0;
                        at = (m >= 0 && m < nm) ? m * 3 + axis : -1;
                        if (DRAWS) {
                            const SrcDesc* S = srcs(desc) + R->src0 + sl;
                            const float u0 = static_cast<float>((S->pos[axis] - R->centre[axis]) / S->d0);
                            extra += part[kPartPos + axis] - part[kPartD0] * u0;
                        }
                    } else if (o < n_mic3 + n_src3) {
                        const bool mine = (o - n_mic3) / 3 == sl;
                        at = mine ? kPartSrc + axis : -1;
                        if (DRAWS && mine) extra += part[kPartD0];
                    } else {
                        at = kPartR;
                    }
                    const float v = part[max(at, 0)];
                    sum += at >= 0 ? v : 0.0f;
                }
            }
        }
        if (o < n_mic3) {
            if (DRAWS) sum += extra / static_cast<float>(R->n_mic);
            if (grad_mic) grad_mic[3 * R->mic0 + o] = sum;
        } else if (o < n_mic3 + n_src3) {
            if (DRAWS) {
                const SrcDesc* S = srcs(desc) + R->src0 + (o - n_mic3) / 3;
                sum += extra * static_cast<float>((S->pos[axis] - R->centre[axis]) / S->d0);
            }
            if (grad_src) grad_src[3 * R->src0 + (o - n_mic3)] = sum;
        } else if (o < n_out) {
            if (grad_r) grad_r[b] = sum;
        }
    }
}

// Backward: per item, dL/dh of the tile core is staged in LDS and every
// (row, microphone) pair of the item's delay range gathers s0 and s1 against
// it; per-thread sums reduce in a fixed two-stage order into the item's
// partials.  The last item of a room to finish (a per-room count) sums the
// room's partials in the plan's order, so the gradients are bitwise
// reproducible whatever the schedule.  Dynamic LDS: max(tile, (NV + 1) NT
// floats), NV = bwd_values(DRAWS).
//
// DRAWS: the images move with the inputs (Eq. 4-6, the Philox variates held
// fixed).  Image i sits at centre + D_i dir_i with D_i = d0 + t_i (cT - d0),
// so with w = dL/dpos_i of a pair (minus the microphone's term) each pair also
// adds w to the item's position sum and (dir_i . w)(1 - t_i) + dL/dg_i
// dg_i/dd0 to its dL/dd0, dL/dg_i = ln(r) s0, and dL/dg_i dg_i/dr to dL/dr.
// dg/dd0 and dg/dr follow Eq. 6 with RR = RR_max(d0, r) of Eq. 5: inside the
// clamp 2 (D/cT^2)(RR - 1)(1 - t) + (D/cT)^2 dRR/dd0 - tau p DR^tau t cT /
// (D d0) and (D/cT)^2 dRR/dr, where p DR^tau = g - 1 - (D/cT)^2 (RR - 1) is
// recovered from the row's g; dRR/dd0 and dRR/dr on the top clamp (g = RR),
// 0 on the bottom one (g = 1).  The direct path (row 0) does not move this way.
template <bool DRAWS>
constexpr int bwd_values() { return DRAWS ? 11 : 7; }

template <int NT, int WPE, bool DRAWS>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE)))
backward_kernel(const void* __restrict__ desc, const double* __restrict__ mic, const double* __restrict__ r_in,
                const float* __restrict__ gout, const double* __restrict__ sorted, const int* __restrict__ bucket_off,
                const int* __restrict__ row0_slot, int* __restrict__ room_done, float* __restrict__ partials,
                int* __restrict__ counters, float* __restrict__ grad_mic, float* __restrict__ grad_src,
                float* __restrict__ grad_r, int lds_words) {
    extern __shared__ float tile[];
    __shared__ int s_item, s_last;
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
        const int mg = c.w.n_mic;
        // Row stride of the staged tile.  The lanes of one image (one per
        // microphone, nearly equal delays) read their rows at the same offset;
        // where the LDS leaves room, rows start about 32 / mg banks apart so
        // that those lanes fall in different banks.
        int stride = c.rowlen;
        {
            const int padded = c.rowlen + (((32 + mg / 2) / mg - c.rowlen) & (kLdsBanks - 1));
            if (mg * padded <= lds_words) stride = padded;
        }
        // dL/dh of the tile core; zero in the halo and beyond T, so that each
        // pair counts only the taps of this tile
        for (int m = 0; m < mg; ++m) {
            const float* g = gout + c.out_off +
                             (static_cast<int64_t>(c.s_local) * c.n_mic_room + c.w.mic0 + m) * c.T;
            for (int k = tid; k < c.rowlen; k += NT) {
                const int n = c.w.t0 - kHalo + k;
                const bool core = k >= kHalo && k < kHalo + c.w.len && n < c.T;
                tile[m * stride + k] = core ? g[n] : 0.0f;
            }
        }
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
        const double4* rows = reinterpret_cast<const double4*>(sorted) + c.img_off + lo;
        const int n_list = hi - lo;
        const int row0 = row0_slot[c.w.src] - lo;   // the direct path, if in range
        const int ipp = NT / mg;
        const int my_m = tid % mg, my_slot = tid / mg;
        const double* mq = mic + 3 * (c.mic0_glob + my_m);
        const double mx = mq[0], my = mq[1], mz = mq[2];
        const float* row = tile + my_m * stride;
        const int shift = kHalo - kHalf - c.w.t0;
        const float fsc = static_cast<float>(c.fs_over_c);
        const float inv_r = static_cast<float>(1.0 / c.r);
        float gmx = 0.f, gmy = 0.f, gmz = 0.f, gsx = 0.f, gsy = 0.f, gsz = 0.f, gr = 0.f;
        // through the draws: per-source constants and the sums over images
        float wx = 0.f, wy = 0.f, wz = 0.f, gd0 = 0.f;
        float d0f = 0.f, inv_span = 0.f, inv_ct = 0.f, rrm1 = 0.f, lnr = 0.f, drr_dd0 = 0.f, drr_dr = 0.f,
              rrf = 0.f, tau_ct_d0 = 0.f;
        if (DRAWS) {
            const SrcDesc* S = srcs(desc) + c.w.src;
            const double ln_r = log(c.r);
            const bool rr_free = S->rrmax > 1.0;   // RR_max not clamped to 1
            d0f = static_cast<float>(S->d0);
            inv_span = static_cast<float>(1.0 / (S->ct - S->d0));
            inv_ct = static_cast<float>(1.0 / S->ct);
            rrf = static_cast<float>(S->rrmax);
            rrm1 = static_cast<float>(S->rrmax - 1.0);
            lnr = static_cast<float>(ln_r);
            drr_dd0 = rr_free ? static_cast<float>(-1.0 / (S->d0 * ln_r)) : 0.f;
            drr_dr = rr_free ? static_cast<float>(-S->rrmax / (c.r * ln_r)) : 0.f;
            const double tau = H->tau_code == kTauQuarter ? 0.25 : H->tau_code == kTauHalf ? 0.5 : 1.0;
            tau_ct_d0 = static_cast<float>(tau * S->ct / S->d0);
        }
        __syncthreads();
        if (my_slot < ipp && my_slot < n_list) {
            int e = my_slot;
            double4 nxt = rows[e];
            while (e < n_list) {
                const double4 cur = nxt;
                const int ce = e;
                e += ipp;
                if (e < n_list) nxt = rows[e];   // prefetch the next pair's row
                const Pair P = pair_setup(cur.x, cur.y, cur.z, mx, my, mz, c.fs_over_c, render_row_amp(cur.w));
                const int b0 = P.k + shift;
                if (b0 < 0 || b0 + kTaps > c.rowlen) continue;
                const float cpd = cospi_small(P.dl);
                const float Ac = P.A * cpd;
                const float S2 = (2.0f * kPiF / 81.0f) * P.S;
                const float v0 = P.A * P.sinc * (P.cy * P.cy);
                // A P'(-dl): sinc'(-dl) w + sinc(dl) w'(-dl), w'(-dl) = (2 pi/81) sy cy
                const float dp0 =
                    P.A * (-dsinc_small(P.dl) * (P.cy * P.cy) + P.sinc * (2.0f * kPiF / 81.0f) * P.sy * P.cy);
                float s0 = 0.f, s1 = 0.f;
                bwd_taps(std::make_integer_sequence<int, kTaps>{}, row + b0, P.cy, P.sy, P.dl, P.S, Ac, S2, v0, dp0,
                         s0, s1);
                const float q = __builtin_fmaf(fsc, s1, s0 / P.D);
                gmx = __builtin_fmaf(P.ux, q, gmx);
                gmy = __builtin_fmaf(P.uy, q, gmy);
                gmz = __builtin_fmaf(P.uz, q, gmz);
                const float g = render_row_g(cur.w);
                if (ce == row0) {
                    gsx -= P.ux * q;
                    gsy -= P.uy * q;
                    gsz -= P.uz * q;
                } else if (DRAWS) {
                    const float ex = static_cast<float>(cur.x - c.cx), ey = static_cast<float>(cur.y - c.cy),
                                ez = static_cast<float>(cur.z - c.cz);
                    const float Dc = __builtin_sqrtf(ex * ex + ey * ey + ez * ez);
                    const float t = (Dc - d0f) * inv_span;
                    // dir . dL/dpos = -q (u . (pos - centre)) / D
                    const float wd = -q * ((P.ux * ex + P.uy * ey + P.uz * ez) / Dc);
                    wx -= P.ux * q;
                    wy -= P.uy * q;
                    wz -= P.uz * q;
                    float dg_dd0 = 0.f, dg_dr = 0.f;
                    if (g >= rrf) {
                        dg_dd0 = drr_dd0;
                        dg_dr = drr_dr;
                    } else if (g > 1.0f) {
                        const float sr = Dc * inv_ct;                      // D / cT
                        const float pdr = (g - 1.0f) - (sr * sr) * rrm1;   // p DR^tau
                        dg_dd0 = 2.0f * sr * inv_ct * rrm1 * (1.0f - t) + (sr * sr) * drr_dd0 -
                                 tau_ct_d0 * pdr * t / Dc;
                        dg_dr = (sr * sr) * drr_dr;
                    }
                    const float lg = lnr * s0;   // dL/dg of the pair
                    gd0 += wd * (1.0f - t) + lg * dg_dd0;
                    gr = __builtin_fmaf(lg, dg_dr, gr);
                }
                gr = __builtin_fmaf(g * inv_r, s0, gr);
            }
        }
        __syncthreads();
        // two-stage fixed-order reduction.  Tasks: (microphone, axis) over
        // the slots of that microphone, then source (3 axes), r and (DRAWS)
        // the position sum (3 axes) and dL/dd0 over all threads; each task in
        // NC chunks, then the chunk sums in order.
        constexpr int NV = bwd_values<DRAWS>();
        float* red = tile;                 // NT x NV
        float* red2 = tile + NV * NT;      // n_task x NC
        red[tid * NV + 0] = gmx;
        red[tid * NV + 1] = gmy;
        red[tid * NV + 2] = gmz;
        red[tid * NV + 3] = gsx;
        red[tid * NV + 4] = gsy;
        red[tid * NV + 5] = gsz;
        red[tid * NV + 6] = gr;
        if (DRAWS) {
            red[tid * NV + 7] = wx;
            red[tid * NV + 8] = wy;
            red[tid * NV + 9] = wz;
            red[tid * NV + 10] = gd0;
        }
        const int n_task = 3 * mg + NV - 3;
        const int NC = max(1, min(NT / n_task, NT / 8));
        __syncthreads();
        if (tid < n_task * NC) {
            const int task = tid / NC, ch = tid % NC;
            float sum = 0.f;
            if (task < 3 * mg) {            // microphone task: threads slot * mg + m
                const int m = task / 3, k = task % 3;
                const int s_lo = (ipp * ch) / NC, s_hi = (ipp * (ch + 1)) / NC;
                for (int sl = s_lo; sl < s_hi; ++sl) sum += red[(sl * mg + m) * NV + k];
            } else {                        // per-item tasks: every thread
                const int k = 3 + (task - 3 * mg), n = ipp * mg;
                const int t_lo = (n * ch) / NC, t_hi = (n * (ch + 1)) / NC;
                for (int t = t_lo; t < t_hi; ++t) sum += red[t * NV + k];
            }
            red2[tid] = sum;
        }
        __syncthreads();
        float* part = partials + static_cast<int64_t>(item) * kPartialStride;
        if (tid < n_task) {
            float sum = 0.f;
            for (int ch = 0; ch < NC; ++ch) sum += red2[tid * NC + ch];
            part[tid < 3 * mg ? tid : kPartSrc + (tid - 3 * mg)] = sum;
        }
        // completion of the room: after the barrier one release fence
        // publishes the item's partials and the item is counted; the last
        // item of the room acquires and sums the room.  (Release and acquire
        // fences, not full ones: an acquire at device scope invalidates the
        // L2 of the XCD, so only the summing workgroup takes it.)
        __syncthreads();
        if (tid == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            s_last = atomicAdd(&room_done[c.room], 1) == rooms(desc)[c.room].n_item - 1;
        }
        __syncthreads();
        if (s_last) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            finalize_room<NT, DRAWS>(desc, c.room, partials, grad_mic, grad_src, grad_r, reinterpret_cast<int*>(tile),
                              lds_words);
            if (tid == 0) atomicExch(&room_done[c.room], 0);
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

// Early-reverberation windows (Eq. 9): blocks over (window chunk, room,
// channel of the room), threads along the window.
__global__ void __launch_bounds__(256) early_kernel(const void* __restrict__ desc, const double* __restrict__ mic,
                                                    const double* __restrict__ src, const float* __restrict__ out,
                                                    float* __restrict__ early, int32_t* __restrict__ start) {
    const DescHeader* H = hdr(desc);
    for (int b = blockIdx.y; b < H->n_rooms; b += gridDim.y) {
        const RoomDesc* R = rooms(desc) + b;
        const int n_chan = R->n_src * R->n_mic;
        const int width = R->early_pre + R->early_post + 1;
        for (int local = blockIdx.z; local < n_chan; local += gridDim.z) {
            const int s = local / R->n_mic, m = local % R->n_mic;
            const int64_t first = early_first(R, src + 3 * (R->src0 + s), mic + 3 * (R->mic0 + m));
            const float* h = out + R->out_off + static_cast<int64_t>(local) * R->T;
            float* e = early + R->early_off + static_cast<int64_t>(local) * width;
            for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < width; j += gridDim.x * blockDim.x) {
                const int64_t n = first + j;
                e[j] = (n >= 0 && n < R->T) ? h[n] : 0.0f;
            }
            if (start && blockIdx.x == 0 && threadIdx.x == 0) start[R->chan0 + local] = static_cast<int32_t>(first);
        }
    }
}

// ---------------------------------------------------------------------------
// Multi-rate chain after the render (Sec. II): 80 Hz high-pass at r_l fs, then
// decimation by r_l.
// ---------------------------------------------------------------------------
// High-pass y[n] = b0 (x[n] - 2 x[n-1] + x[n-2]) - a1 y[n-1] - a2 y[n-2] (FP64),
// from rest, evaluated in parallel and exactly: the deviation d = y - x of the
// output state, (y[s-1] - x[s-1], y[s-2] - x[s-2]), is found at every
// sub-chunk start s (kHpSub samples apart) before the decimation runs, which
// then runs the recurrence from those states over just the samples it needs.
// The deviations come from partial runs: a span filtered with its true input
// history and its output history set equal to that input history (deviation
// 0) ends at deviation e; the true run, starting at deviation d, differs from
// it by the unforced response of d, so it ends at e + phi d (phi the span's
// state transition).  hp_chunk_end_kernel: partial runs over the sub-chunks,
// one thread each, combined in order within each chunk into the chunk's
// partial run: its deviation p_j at sub-chunk j's start and e(k) at its end;
// hp_carry_kernel: one thread per channel carries the chunk starts, d(k + 1) =
// e(k) + phi d(k); sub-chunk j of chunk k then starts at p_j + phi_sub[j] d(k).

// Raw buffer view of n floats at p: loads at byte offsets >= 4 n return 0
// (range checking of untyped buffer accesses with stride 0; word 3 selects
// the 32-bit data format).  The check covers the VGPR offset and the
// instruction's immediate offset but not the SGPR offset, so every access
// passes its whole offset in the VGPR operand; offsets before the start are
// given as 2^31 bytes, past any view.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_view(const float* p, int n) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(p), static_cast<short>(0), 4 * n, 0x00020000);
}
// (The b32 builtin moves 32-bit integers: the floats go through a bit cast.)
__device__ __forceinline__ float view_load(__amdgpu_buffer_rsrc_t v, int64_t i) {
    const int off = i >= 0 ? static_cast<int>(4 * i) : INT32_MIN;
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(v, off, 0, 0));
}

// One step of the high-pass in direct form, the feedback as FMAs: the
// dependence from one output to the next is a single FMA.
__device__ __forceinline__ double hp_step(double xn, double& x1, double& x2, double& y1, double& y2, double b0,
                                          double a1, double a2) {
    const double yn = __builtin_fma(-a1, y1, __builtin_fma(-a2, y2, b0 * ((xn - 2.0 * x1) + x2)));
    x2 = x1;
    x1 = xn;
    y2 = y1;
    y1 = yn;
    return yn;
}

// Deviation at the end of the partial run over one sub-chunk (32 samples in
// registers, input history x1, x2).
__device__ __forceinline__ double2 hp_sub_partial(const float (&xr)[kHpSub], double x1, double x2, double b0,
                                                  double a1, double a2) {
    double y1 = x1, y2 = x2;
#pragma unroll
    for (int i = 0; i < kHpSub; ++i) hp_step(xr[i], x1, x2, y1, y2, b0, a1, a2);
    return double2{y1 - x1, y2 - x2};
}

// LDS word of sample w of a staged run: one pad word after every 32, so that
// thread t's sub-chunk (words 33 t ..) and consecutive samples both spread
// over the banks.
__device__ __forceinline__ int hp_word(int w) { return w + (w >> 5); }

constexpr int kHpSubPerChunk = kHpChunk / kHpSub;        // 8
constexpr int kHpEndGrid = 1024;                         // persistent workgroups of hp_chunk_end_kernel
constexpr int kHpEndThreads = kHpEndChunks * kHpSubPerChunk;
static_assert(kHpEndThreads == 256 && kHpSub == 32, "one sub-chunk per thread, 32 chunks per block");

// Partial deviations of every chunk: a task is a block of 32 consecutive
// chunks of a channel (8192 samples, loaded coalesced into LDS); thread =
// sub-chunk; the sub-chunk end deviations e_j are combined in order by one
// thread per chunk, p_0 = 0, p_(j+1) = e_j + phi_sub[1] p_j: p_j to sub (one
// per sub-chunk), p_8 = e(k) to zend.  The grid is persistent over the plan's
// task list: while a block runs its recursion, the next block's samples are
// already in flight, so the loads never wait on a descriptor chain or an idle
// workgroup.
__global__ void __launch_bounds__(kHpEndThreads) hp_chunk_end_kernel(const void* __restrict__ desc,
                                                                     const float* __restrict__ x,
                                                                     double* __restrict__ zend,
                                                                     double2* __restrict__ sub) {
    constexpr int kSamples = kHpEndChunks * kHpChunk;
    constexpr int kPer = kSamples / kHpEndThreads;     // samples per thread and block
    __shared__ float xs[kSamples + kSamples / 32];
    __shared__ double2 es[kHpEndThreads];
    const DescHeader* H = hdr(desc);
    const HpTask* tasks = hp_tasks(desc);
    const int n_tasks = H->n_hp_tasks;
    const int tid = threadIdx.x;
    int t = blockIdx.x;
    if (t >= n_tasks) return;
    // a block's samples in registers, coalesced (thread 0 also the two before
    // the block: the input history of its first sub-chunk; 0 before the start)
    float v[kPer];
    float h1 = 0.0f, h2 = 0.0f;
    auto fetch = [&](int task) {
        const HpTask k = tasks[task];
        const RoomDesc* R = rooms(desc) + k.room;
        const __amdgpu_buffer_rsrc_t xv = buffer_view(x + R->out_off + static_cast<int64_t>(k.chan) * R->T, R->T);
        const int64_t s0 = static_cast<int64_t>(k.blk) * kSamples;
#pragma unroll
        for (int q = 0; q < kPer; ++q) v[q] = view_load(xv, s0 + tid + kHpEndThreads * q);
        if (tid == 0) {
            h1 = view_load(xv, s0 - 1);
            h2 = view_load(xv, s0 - 2);
        }
    };
    fetch(t);
    for (;;) {
        const HpTask k = tasks[t];
        const RoomDesc* R = rooms(desc) + k.room;
        const int c0 = k.blk * kHpEndChunks;
        __syncthreads();   // the previous block's reads of xs and es are done
#pragma unroll
        for (int q = 0; q < kPer; ++q) xs[hp_word(tid + kHpEndThreads * q)] = v[q];
        const double hx1 = h1, hx2 = h2;
        __syncthreads();
        const int tn = t + static_cast<int>(gridDim.x);
        if (tn < n_tasks) fetch(tn);   // the next block streams in during this one's recursion
        const double b0 = R->hp_b0, a1 = R->hp_a1, a2 = R->hp_a2;
        const int w0 = kHpSub * tid;
        double x1, x2;
        if (tid == 0) {
            x1 = hx1;
            x2 = hx2;
        } else {
            x1 = xs[hp_word(w0 - 1)];
            x2 = xs[hp_word(w0 - 2)];
        }
        float xr[kHpSub];
#pragma unroll
        for (int i = 0; i < kHpSub; ++i) xr[i] = xs[hp_word(w0 + i)];
        es[tid] = hp_sub_partial(xr, x1, x2, b0, a1, a2);
        __syncthreads();
        const int64_t ci0 = R->chunk0 + static_cast<int64_t>(k.chan) * R->n_chunks + c0;   // the block's first chunk
        const int c = c0 + tid;
        if (tid < kHpEndChunks && c < R->n_chunks) {
            const double* ph = R->phi_sub[1];
            double d0 = 0.0, d1 = 0.0;
            for (int j = 0; j < kHpSubPerChunk; ++j) {
                const double2 e = es[kHpSubPerChunk * tid + j];
                es[kHpSubPerChunk * tid + j] = double2{d0, d1};
                const double n0 = e.x + (ph[0] * d0 + ph[1] * d1);
                const double n1 = e.y + (ph[2] * d0 + ph[3] * d1);
                d0 = n0;
                d1 = n1;
            }
            zend[2 * (ci0 + tid)] = d0;
            zend[2 * (ci0 + tid) + 1] = d1;
        }
        __syncthreads();
        if (c0 + tid / kHpSubPerChunk < R->n_chunks) sub[kHpSubPerChunk * ci0 + tid] = es[tid];
        if (tn >= n_tasks) break;
        t = tn;
    }
}

// Deviation at every chunk start, one thread per channel, chunk after chunk:
// d(0) = 0, d(k + 1) = e(k) + phi d(k).
__global__ void __launch_bounds__(64) hp_carry_kernel(const void* __restrict__ desc, const double* __restrict__ zend,
                                                      double* __restrict__ init) {
    const DescHeader* H = hdr(desc);
    for (int b = blockIdx.x; b < H->n_rooms; b += gridDim.x) {
        const RoomDesc* R = rooms(desc) + b;
        const double p0 = R->phi[0], p1 = R->phi[1], p2 = R->phi[2], p3 = R->phi[3];
        for (int local = threadIdx.x; local < R->n_src * R->n_mic; local += blockDim.x) {
            const int64_t c0 = R->chunk0 + static_cast<int64_t>(local) * R->n_chunks;
            double s0 = 0.0, s1 = 0.0;
            // the partial end deviations of kCarryAhead chunks are loaded together, so
            // that the recurrence waits for memory once per group of chunks
            constexpr int kCarryAhead = 32;
            for (int k0 = 0; k0 < R->n_chunks; k0 += kCarryAhead) {
                double2 z[kCarryAhead];
#pragma unroll
                for (int j = 0; j < kCarryAhead; ++j) {
                    const int k = min(k0 + j, R->n_chunks - 1);
                    z[j] = reinterpret_cast<const double2*>(zend)[c0 + k];
                }
#pragma unroll
                for (int j = 0; j < kCarryAhead; ++j) {
                    const int k = k0 + j;
                    if (k < R->n_chunks) {
                        init[2 * (c0 + k)] = s0;
                        init[2 * (c0 + k) + 1] = s1;
                        const double n0 = z[j].x + (p0 * s0 + p1 * s1);
                        const double n1 = z[j].y + (p2 * s0 + p3 * s1);
                        s0 = n0;
                        s1 = n1;
                    }
                }
            }
        }
    }
}


// Decimation by r_l (Sec. II): out[n] = sum_j y[j] P((n r_l - j) / r_l), the
// 81-tap Hann-windowed sinc in units of fs (2 half + 1 taps, half = ceil(40.5
// r_l) - 1), y the high-passed intermediate signal (zero outside [0, T_l)).
// A block of 256 outputs is a 16 x 16 tile D[i][b] = out[n0 + 16 b + i] =
// sum_q W[i][q] Y[q][b] with Y[q][b] = y[(n0 + 16 b) r_l - half - pad + q] and
// W[i][q] = k[i r_l + half + pad - q] (zero outside |u| <= half): a Toeplitz
// product with the same W for every block, on the matrix cores
// (v_mfma_f32_16x16x32_f16; pad makes half + pad a multiple of 32, so that
// every tile's span starts on a sub-chunk boundary and every 8-element operand
// on a 16-byte boundary).  Operands are fp16 pairs hi + lo (the inputs scaled
// by a power of two per tile so that the largest is near 2^14), products
// hi*hi + hi*lo + lo*hi accumulated in FP32.

__host__ __device__ constexpr int dm_half(int rl) { return (81 * rl + 1) / 2 - 1; }   // ceil(40.5 r_l) - 1
__host__ __device__ constexpr int dm_pad(int rl) { return (32 - dm_half(rl) % 32) % 32; }
__host__ __device__ constexpr int dm_steps(int rl) {
    return (dm_pad(rl) + 15 * rl + 2 * dm_half(rl) + 1 + 31) / 32;
}
__host__ __device__ constexpr bool dm_steps_fit() {
    for (int rl = 1; rl <= kMaxRl; ++rl)
        if (dm_steps(rl) > kDmMaxSteps) return false;
    return true;
}
static_assert(dm_steps_fit(), "fragment table too small for an r_l");

// Window element e sits in word e + 4 (e / 32): four pad words after every 32
// elements spread the 16 columns of an operand read (16 r_l elements apart)
// over the LDS banks; pairs, runs of 8 and sub-chunks stay inside one run of
// 32 (a sub-chunk is words 36 g .. 36 g + 31).
__device__ __forceinline__ int dm_word(int e) { return e + 4 * (e >> 5); }
__host__ __device__ constexpr int dm_span(int rl) { return (kDmOut - 1) * rl + 2 * dm_half(rl) + 1 + dm_pad(rl); }
// A tile stages the window from the start of the chunk holding its span's
// first sample: at most kHpChunk - kHpSub samples before the span, the span,
// the rest of its last sub-chunk and one sub-chunk of zeros (operand reads
// end at most 31 elements past the span).
__host__ __device__ constexpr int dm_window(int rl) { return (kHpChunk - kHpSub) + dm_span(rl) + 2 * kHpSub; }
// (at least the four waves' partial tiles: 16 x 256 floats)
__host__ __device__ constexpr int dm_lds_words(int rl) {
    return dm_window(rl) + 4 * ((dm_window(rl) + 31) / 32) > 16 * 256 ? dm_window(rl) + 4 * ((dm_window(rl) + 31) / 32)
                                                                        : 16 * 256;
}

// The W fragments of every r_l the plan uses: workgroup (r_l - 1, step), lane l
// (row i = l mod 16, columns 8 (l / 16) .. + 7 of each step); P(u / r_l) in
// FP64, rounded to FP32, then split into fp16 hi and lo.
__global__ void __launch_bounds__(64) dec_frag_kernel(const void* __restrict__ desc, uint32_t* __restrict__ frag) {
    const DescHeader* H = hdr(desc);
    const int rl = blockIdx.x + 1, st = blockIdx.y;
    __shared__ int used;
    if (threadIdx.x == 0) used = 0;
    __syncthreads();
    for (int b = threadIdx.x; b < H->n_rooms; b += blockDim.x)
        if (static_cast<int>(rooms(desc)[b].rl) == rl) used = 1;
    __syncthreads();
    const int half = dm_half(rl), pad = dm_pad(rl);
    if (!used || st >= dm_steps(rl)) return;
    const int l = threadIdx.x, i = l % 16;
    uint32_t* f = frag + static_cast<int64_t>(rl - 1) * kDmFragWords;
    {
        uint32_t hw[4] = {0u, 0u, 0u, 0u}, lw[4] = {0u, 0u, 0u, 0u};
        for (int e = 0; e < 8; ++e) {
            const int q = 32 * st + 8 * (l / 16) + e;
            const int u = i * rl + half + pad - q;
            float c = 0.0f;
            if (u >= -half && u <= half) {
                const double xv = static_cast<double>(u) / rl;
                double sp, cp, sw, cw;
                sincospi_d(xv, &sp, &cp);
                sincospi_d(2.0 * xv / 81.0, &sw, &cw);
                const double sinc = u == 0 ? 1.0 : sp / (3.141592653589793 * xv);
                c = static_cast<float>(sinc * 0.5 * (1.0 + cw));
            }
            const _Float16 h = static_cast<_Float16>(c);
            const _Float16 o = static_cast<_Float16>(c - static_cast<float>(h));
            hw[e / 2] |= static_cast<uint32_t>(__builtin_bit_cast(uint16_t, h)) << (16 * (e & 1));
            lw[e / 2] |= static_cast<uint32_t>(__builtin_bit_cast(uint16_t, o)) << (16 * (e & 1));
        }
        for (int w = 0; w < 4; ++w) {
            f[(st * 2 + 0) * 256 + 4 * l + w] = hw[w];
            f[(st * 2 + 1) * 256 + 4 * l + w] = lw[w];
        }
    }
}

// Start state of sub-chunk g of a decimation window: input history x1, x2,
// the chunk's partial deviation p at the sub-chunk and the chunk's start
// deviation i (0 before the signal, and for chunk 0).
struct DmStart {
    float x1, x2;
    double2 p, i;
};
__device__ __forceinline__ DmStart dm_start_load(__amdgpu_buffer_rsrc_t xv, const double2* __restrict__ sub,
                                                 const double* __restrict__ init, const RoomDesc* R, int64_t ci0,
                                                 int64_t kf, int64_t wb, int g, int n_sub) {
    DmStart r{0.0f, 0.0f, double2{0.0, 0.0}, double2{0.0, 0.0}};
    if (g >= n_sub) return r;
    const int64_t s = wb + static_cast<int64_t>(kHpSub) * g;
    const int64_t k = kf + g / kHpSubPerChunk;
    r.x1 = view_load(xv, s - 1);
    r.x2 = view_load(xv, s - 2);
    if (k >= 0 && k < R->n_chunks) {
        r.p = sub[kHpSubPerChunk * (ci0 + k) + g % kHpSubPerChunk];
        if (k > 0) r.i = reinterpret_cast<const double2*>(init)[ci0 + k];
    }
    return r;
}

// One workgroup per (tile of kDmOut outputs, room, channel).  Staging: the
// window from the start of chunk k_first (the chunk holding the span's first
// sample) is loaded coalesced into LDS; thread t then takes sub-chunks t, t +
// 256, ... (32 samples each), starts at deviation p_j + phi_sub[j] d(k) with
// its input history from memory, and runs the recurrence over its samples,
// writing y (0 outside [0, T_l)) over them.  The span is scaled and converted
// in place to fp16 halves: each group of 8 elements (8-aligned) becomes four
// words of hi halves, then four of lo halves, so that an operand's hi and lo
// parts are one 16-byte read each.  Products: the K steps are dealt to
// the four waves in turn; a wave applies each filter fragment it loads to all
// four 256-output blocks (four independent accumulators), and the partial
// tiles are summed through LDS in wave order.
__global__ void __launch_bounds__(kDmThreads) __attribute__((amdgpu_waves_per_eu(4))) decimate_mfma_kernel(const void* __restrict__ desc,
                                                                   const float* __restrict__ x,
                                                                   const double* __restrict__ init,
                                                                   const double2* __restrict__ sub,
                                                                   const uint32_t* __restrict__ frag,
                                                                   float* __restrict__ out) {
    extern __shared__ u32x4 span_v[];
    float* span = reinterpret_cast<float*>(span_v);
    __shared__ int s_max;   // largest |y| of the tile's span, as float bits
    static_assert(kHpSub == 32 && kDmBlocks * 64 == kDmThreads, "one wave per block");
    constexpr int kLoads = 8;   // window samples per thread in flight (4 waves per SIMD without spills)
    const DescHeader* H = hdr(desc);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int col = lane & 15, grp = lane >> 4;
    for (int b = blockIdx.y; b < H->n_rooms; b += gridDim.y) {
        const RoomDesc* R = rooms(desc) + b;
        const int rl = static_cast<int>(R->rl);
        const int half = dm_half(rl), pad = dm_pad(rl), steps = dm_steps(rl), span_len = dm_span(rl);
        const double b0 = R->hp_b0, a1 = R->hp_a1, a2 = R->hp_a2;
        const int T = R->T;
        const uint32_t* fr = frag + static_cast<int64_t>(rl - 1) * kDmFragWords;
        const int n_tiles = (R->T_out + kDmOut - 1) / kDmOut;
        for (int local = blockIdx.z; local < R->n_src * R->n_mic; local += gridDim.z) {
            const __amdgpu_buffer_rsrc_t xv = buffer_view(x + R->out_off + static_cast<int64_t>(local) * T, T);
            const int64_t ci0 = R->chunk0 + static_cast<int64_t>(local) * R->n_chunks;
            for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
                const int n0 = tile * kDmOut;
                const int64_t jb = static_cast<int64_t>(n0) * rl - half - pad;   // span start (multiple of 32)
                const int64_t kf = jb >> 8;                                      // k_first (kHpChunk = 256)
                const int64_t wb = kf * kHpChunk;                                // window start
                const int woff = static_cast<int>(jb - wb);
                const int n_sub = (woff + span_len + kHpSub - 1) / kHpSub;
                const int n_el = n_sub * kHpSub;
                // the first sub-chunk's start state loads while the window lands
                DmStart ss = dm_start_load(xv, sub, init, R, ci0, kf, wb, tid, n_sub);
                __syncthreads();   // the previous tile's reads are done
                if (tid == 0) s_max = 0;
                // coalesced load of the window
                for (int w0 = 0; w0 < n_el; w0 += kLoads * kDmThreads) {
                    float v[kLoads];
#pragma unroll
                    for (int u = 0; u < kLoads; ++u) {
                        const int w = w0 + tid + kDmThreads * u;
                        v[u] = w < n_el ? view_load(xv, wb + w) : 0.0f;
                    }
#pragma unroll
                    for (int u = 0; u < kLoads; ++u) {
                        const int w = w0 + tid + kDmThreads * u;
                        if (w < n_el) span[dm_word(w)] = v[u];
                    }
                }
                for (int w = n_el + tid; w < n_el + kHpSub; w += kDmThreads) span[dm_word(w)] = 0.0f;
                __syncthreads();
                float vmax = 0.0f;
                for (int g = tid; g < n_sub; g += kDmThreads) {
                    if (g != tid) ss = dm_start_load(xv, sub, init, R, ci0, kf, wb, g, n_sub);
                    const int64_t s = wb + static_cast<int64_t>(kHpSub) * g;   // first sample of the sub-chunk
                    const double* ph = R->phi_sub[g % kHpSubPerChunk];
                    double x1 = ss.x1, x2 = ss.x2;
                    const double d0 = ss.p.x + (ph[0] * ss.i.x + ph[1] * ss.i.y);
                    const double d1 = ss.p.y + (ph[2] * ss.i.x + ph[3] * ss.i.y);
                    float xr[kHpSub];
                    const f32x4* src = reinterpret_cast<const f32x4*>(span + dm_word(kHpSub * g));
#pragma unroll
                    for (int i = 0; i < kHpSub / 4; ++i) {
                        const f32x4 q = src[i];
                        xr[4 * i] = q.x;
                        xr[4 * i + 1] = q.y;
                        xr[4 * i + 2] = q.z;
                        xr[4 * i + 3] = q.w;
                    }
                    double y1 = x1 + d0, y2 = x2 + d1;
                    const bool inside = s >= 0 && s + kHpSub <= T;
#pragma unroll
                    for (int i = 0; i < kHpSub; ++i) {
                        const float yv = static_cast<float>(hp_step(xr[i], x1, x2, y1, y2, b0, a1, a2));
                        xr[i] = inside || (s + i >= 0 && s + i < T) ? yv : 0.0f;
                    }
                    if (kHpSub * g >= woff)
#pragma unroll
                        for (int i = 0; i < kHpSub; ++i) vmax = fmaxf(vmax, fabsf(xr[i]));
                    f32x4* dst = reinterpret_cast<f32x4*>(span + dm_word(kHpSub * g));
#pragma unroll
                    for (int i = 0; i < kHpSub / 4; ++i) dst[i] = f32x4{xr[4 * i], xr[4 * i + 1], xr[4 * i + 2], xr[4 * i + 3]};
                }
                atomicMax(&s_max, __float_as_int(vmax));
                // the wave's first two steps' filter fragments load during the conversion
                int fl = lane;
                asm volatile("" : "+v"(fl));
                u32x4 ah = u32x4{0u, 0u, 0u, 0u}, al = ah, ahn = ah, aln = ah;   // steps wave and wave + 4
                if (wave < steps) {
                    ah = *reinterpret_cast<const u32x4*>(fr + (wave * 2 + 0) * 256 + 4 * fl);
                    al = *reinterpret_cast<const u32x4*>(fr + (wave * 2 + 1) * 256 + 4 * fl);
                }
                if (wave + kDmBlocks < steps) {
                    ahn = *reinterpret_cast<const u32x4*>(fr + ((wave + kDmBlocks) * 2 + 0) * 256 + 4 * fl);
                    aln = *reinterpret_cast<const u32x4*>(fr + ((wave + kDmBlocks) * 2 + 1) * 256 + 4 * fl);
                }
                __syncthreads();
                // scale: the largest input to ~2^14 (fp16 keeps the lo halves normal)
                const float mx = __int_as_float(s_max);
                const int ex = mx > 0.0f ? max(-100, (__float_as_int(mx) >> 23) - 127) : 0;
                const float sc = __int_as_float((127 + 14 - ex) << 23), inv_sc = __int_as_float((127 - 14 + ex) << 23);
                for (int q = woff / 8 + tid; q < (n_el + kHpSub) / 8; q += kDmThreads) {
                    // elements 8q .. 8q + 7: four words of hi halves, then four of lo halves
                    f32x4* w = reinterpret_cast<f32x4*>(span + dm_word(8 * q));
                    const f32x4 x0 = w[0] * sc, x1 = w[1] * sc;
                    const u32x4 hw = u32x4{pack_f16(x0.x, x0.y), pack_f16(x0.z, x0.w), pack_f16(x1.x, x1.y),
                                           pack_f16(x1.z, x1.w)};
                    const u32x4 lw = u32x4{pack_f16(x0.x - f16_lo_of(hw.x), x0.y - f16_hi_of(hw.x)),
                                           pack_f16(x0.z - f16_lo_of(hw.y), x0.w - f16_hi_of(hw.y)),
                                           pack_f16(x1.x - f16_lo_of(hw.z), x1.y - f16_hi_of(hw.z)),
                                           pack_f16(x1.z - f16_lo_of(hw.w), x1.w - f16_hi_of(hw.w))};
                    reinterpret_cast<u32x4*>(w)[0] = hw;
                    reinterpret_cast<u32x4*>(w)[1] = lw;
                }
                __syncthreads();
                // steps wave, wave + 4, ...: column col of block blk starts at
                // window element woff + (256 blk + 16 col) r_l
                f32x4 acc[kDmBlocks];
#pragma unroll
                for (int blk = 0; blk < kDmBlocks; ++blk) acc[blk] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
                // operand words of step st: dm_word(e + 32 st) = dm_word(e) + 36 st
                const u32x4* bw[kDmBlocks];
#pragma unroll
                for (int blk = 0; blk < kDmBlocks; ++blk)
                    bw[blk] = reinterpret_cast<const u32x4*>(span) +
                              dm_word(woff + (256 * blk + 16 * col) * rl + 8 * grp + 32 * wave) / 4;
                constexpr int kStepWords = 36 * kDmBlocks / 4;   // u32x4 per dealt step
                for (int st = wave; st < steps; st += kDmBlocks) {
                    u32x4 ahf = ahn, alf = aln;   // two steps ahead
                    if (st + 2 * kDmBlocks < steps) {
                        ahf = *reinterpret_cast<const u32x4*>(fr + ((st + 2 * kDmBlocks) * 2 + 0) * 256 + 4 * fl);
                        alf = *reinterpret_cast<const u32x4*>(fr + ((st + 2 * kDmBlocks) * 2 + 1) * 256 + 4 * fl);
                    }
#pragma unroll
                    for (int h = 0; h < kDmBlocks; h += 2) {   // two blocks' operands at a time
                        const u32x4 bh0 = bw[h][0], bl0 = bw[h][1], bh1 = bw[h + 1][0], bl1 = bw[h + 1][1];
                        acc[h] = mfma_16x16x32(ah, bh0, acc[h]);
                        acc[h + 1] = mfma_16x16x32(ah, bh1, acc[h + 1]);
                        acc[h] = mfma_16x16x32(ah, bl0, acc[h]);
                        acc[h + 1] = mfma_16x16x32(ah, bl1, acc[h + 1]);
                        acc[h] = mfma_16x16x32(al, bh0, acc[h]);
                        acc[h + 1] = mfma_16x16x32(al, bh1, acc[h + 1]);
                    }
#pragma unroll
                    for (int blk = 0; blk < kDmBlocks; ++blk) bw[blk] += kStepWords;
                    ah = ahn;
                    al = aln;
                    ahn = ahf;
                    aln = alf;
                }
                __syncthreads();   // every wave is done with the span: it now holds the partial tiles
                f32x4* part = reinterpret_cast<f32x4*>(span);
#pragma unroll
                for (int blk = 0; blk < kDmBlocks; ++blk) part[(wave * kDmBlocks + blk) * 64 + lane] = acc[blk];
                __syncthreads();
                f32x4 sum = part[wave * 64 + lane];
#pragma unroll
                for (int v = 1; v < kDmBlocks; ++v) sum += part[(v * kDmBlocks + wave) * 64 + lane];
                // lane: outputs n .. n + 3 (rows 4 grp .. 4 grp + 3 of column col of block wave)
                float* o = out + R->out2_off + static_cast<int64_t>(local) * R->T_out;
                const int n = n0 + 256 * wave + 16 * col + 4 * grp;
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (n + i < R->T_out) o[n + i] = sum[i] * inv_sc;
            }
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
template <auto Kernel, int Bytes = kMaxDynLdsBytes>
int allow_lds() {
    static int status = [] {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(Kernel),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, Bytes);
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
    int* row0_slot;
    int* room_done;
    double* sorted;
};

RenderWs render_ws(const framrir_plan* plan, void* ws_dev) {
    char* b = static_cast<char*>(ws_dev);
    return RenderWs{reinterpret_cast<int*>(b),
                    reinterpret_cast<float*>(b + plan->ws_scale_off),
                    reinterpret_cast<int*>(b + plan->ws_bucket_off),
                    reinterpret_cast<int*>(b + plan->ws_row0_off),
                    reinterpret_cast<int*>(b + plan->ws_room_off),
                    reinterpret_cast<double*>(b + plan->ws_rows_off)};
}

int launch_prepare(const framrir_plan* plan, const void* desc_dev, double* table_dev, const double* mic_dev,
                   const double* src_dev, const double* r_dev, void* ws_dev, hipStream_t st, bool draw) {
    const RenderWs w = render_ws(plan, ws_dev);
    // preparation (and, for the forward, the draws themselves): one workgroup per source
    const int key_cap = prep_key_cap(plan->header.max_img);
    const int lds = prep_dyn_lds(plan->header.max_img);
    if (draw) {
        if (int rc = allow_lds<prep_kernel<true>, prep_dyn_lds(kMaxImg)>()) return rc;
        hipLaunchKernelGGL(prep_kernel<true>, dim3(plan->header.n_src), dim3(kPrepThreads), lds, st, desc_dev, table_dev,
                           mic_dev, src_dev, r_dev, w.src_scale, w.bucket_off, w.row0_slot, w.room_done, w.sorted,
                           key_cap);
    } else {
        if (int rc = allow_lds<prep_kernel<false>, prep_dyn_lds(kMaxImg)>()) return rc;
        hipLaunchKernelGGL(prep_kernel<false>, dim3(plan->header.n_src), dim3(kPrepThreads), lds, st, desc_dev, table_dev,
                           mic_dev, src_dev, r_dev, w.src_scale, w.bucket_off, w.row0_slot, w.room_done, w.sorted,
                           key_cap);
    }
    return check_launch("prep_kernel");
}

int launch_render(const framrir_plan* plan, const void* desc_dev, const double* table_dev, const double* mic_dev,
                  const double* src_dev, const double* r_dev, float* out_dev, void* ws_dev, hipStream_t st,
                  float* early_dev = nullptr, int32_t* start_dev = nullptr) {
    const RenderWs w = render_ws(plan, ws_dev);
    const int lds = plan->launch.lds_bytes;
    const int acc_words = plan->launch.lds_bytes / 4;
    const dim3 grid(plan->grid), block(plan->launch.wg_threads);
    const int key = plan->launch.wg_threads * 16 + plan->launch.waves_per_simd;
    if (plan->launch.render_path == 1) {   // compiled at 4 waves per SIMD only (the plan checks it)
        switch (key) {
#define FR_CASE(NT)                                                                                          \
    case NT * 16 + 4:                                                                                        \
        if (early_dev) {                                                                                     \
            if (int rc = allow_lds<render_moment_kernel<NT, 4, true>, kLdsPerCu - kMomStaticLds>()) return rc; \
            hipLaunchKernelGGL((render_moment_kernel<NT, 4, true>), grid, block, lds, st, desc_dev, mic_dev, \
                               src_dev, r_dev, out_dev, w.counters, w.src_scale, w.bucket_off, w.sorted,     \
                               acc_words, early_dev, start_dev);                                             \
        } else {                                                                                             \
            if (int rc = allow_lds<render_moment_kernel<NT, 4, false>, kLdsPerCu - kMomStaticLds>()) return rc; \
            hipLaunchKernelGGL((render_moment_kernel<NT, 4, false>), grid, block, lds, st, desc_dev, mic_dev, \
                               src_dev, r_dev, out_dev, w.counters, w.src_scale, w.bucket_off, w.sorted,     \
                               acc_words, nullptr, nullptr);                                                 \
        }                                                                                                    \
        break;
            FR_CASE(256) FR_CASE(512) FR_CASE(1024)
#undef FR_CASE
            default:
                return fr_fail(FRAMRIR_E_UNSUPPORTED, "launch shape %d threads x %d waves/SIMD not compiled",
                               plan->launch.wg_threads, plan->launch.waves_per_simd);
        }
        return check_launch("render_moment_kernel");
    }
    switch (key) {
#define FR_CASE(NT, WPE)                                                                                     \
    case NT * 16 + WPE:                                                                                      \
        if (early_dev) {                                                                                     \
            if (int rc = allow_lds<render_kernel<NT, WPE, true>, kLdsPerCu - render_static_lds(NT)>()) return rc; \
            hipLaunchKernelGGL((render_kernel<NT, WPE, true>), grid, block, lds, st, desc_dev, table_dev,    \
                               mic_dev, src_dev, r_dev, out_dev, w.counters, w.src_scale, w.bucket_off,     \
                               w.sorted, acc_words, early_dev, start_dev);                                   \
        } else {                                                                                             \
            if (int rc = allow_lds<render_kernel<NT, WPE, false>, kLdsPerCu - render_static_lds(NT)>()) return rc; \
            hipLaunchKernelGGL((render_kernel<NT, WPE, false>), grid, block, lds, st, desc_dev, table_dev,   \
                               mic_dev, src_dev, r_dev, out_dev, w.counters, w.src_scale, w.bucket_off,     \
                               w.sorted, acc_words, nullptr, nullptr);                                       \
        }                                                                                                    \
        break;
        FR_KERNEL_SHAPES(FR_CASE)
#undef FR_CASE
        default:
            return fr_fail(FRAMRIR_E_UNSUPPORTED, "launch shape %d threads x %d waves/SIMD not compiled",
                           plan->launch.wg_threads, plan->launch.waves_per_simd);
    }
    return check_launch("render_kernel");
}

// table_dev may be NULL where the call does not read it (a forward that
// draws, the render of prepared rows).
int check_render_args(const framrir_plan* plan, const void* desc_dev, const double* table_dev, const double* mic_dev,
                      const double* src_dev, const void* out_dev, void* ws_dev, size_t ws_bytes, int64_t need,
                      bool table_required = true) {
    if (!plan || !desc_dev || (table_required && !table_dev) || !mic_dev || !src_dev || !out_dev || !ws_dev)
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
    if (plan && plan->header.multirate)
        return fr_fail(FRAMRIR_E_UNSUPPORTED, "multi-rate plan: use framrir_forward_multirate");
    // (no output buffer: the workspace stands in for it in the check)
    int rc = check_render_args(plan, desc_dev, table_dev, mic_dev, src_dev, ws_dev, ws_dev, ws_bytes,
                               plan ? plan->ws_bytes : 0, draw == 0);
    if (rc) return rc;
    return launch_prepare(plan, desc_dev, table_dev, mic_dev, src_dev, r_dev, ws_dev, static_cast<hipStream_t>(stream),
                          draw != 0);
}

extern "C" int framrir_render_prepared(const framrir_plan* plan, const void* desc_dev, const double* table_dev,
                                       const double* mic_dev, const double* src_dev, const double* r_dev,
                                       float* out_dev, void* ws_dev, size_t ws_bytes, void* stream) {
    if (plan && plan->header.multirate)
        return fr_fail(FRAMRIR_E_UNSUPPORTED, "multi-rate plan: use framrir_forward_multirate");
    int rc = check_render_args(plan, desc_dev, table_dev, mic_dev, src_dev, out_dev, ws_dev, ws_bytes,
                               plan ? plan->ws_bytes : 0, false);
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

// ---------------------------------------------------------------------------
// Allocation-free forward: framrir_forward with its workspace in a static
// device array of the library, for callers that cannot allocate.
// ---------------------------------------------------------------------------
// The array itself; each device that runs the library holds its own copy
// until the process ends.  Host code never passes its name to a kernel (on the
// host the name is only a stand-in): it uses the device address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[FRAMRIR_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxScratchDevices] = {};

// Device address of the current device's scratch, looked up once per device
// (with that device current) and kept.
int current_scratch(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fr_fail(FRAMRIR_E_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxScratchDevices)
        return fr_fail(FRAMRIR_E_UNSUPPORTED, "device %d: at most %d devices", dev, kMaxScratchDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fr_fail(FRAMRIR_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                           hipGetErrorString(e));
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return FRAMRIR_OK;
}

}  // namespace

// Looks up (once) the static scratch of `device`, with that device current;
// called when a handle is created for the device.
int framrir_scratch_setup(int device) {
    int prev = 0;
    hipError_t e = hipGetDevice(&prev);
    if (e != hipSuccess) return fr_fail(FRAMRIR_E_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if ((e = hipSetDevice(device)) != hipSuccess)
        return fr_fail(FRAMRIR_E_DEVICE, "hipSetDevice(%d): %s", device, hipGetErrorString(e));
    void* p = nullptr;
    const int rc = current_scratch(&p);
    (void)hipSetDevice(prev);
    return rc;
}

extern "C" int framrir_forward_noalloc(const framrir_plan* plan, const void* desc_dev, double* table_dev,
                                       const double* mic_dev, const double* src_dev, const double* r_dev,
                                       float* out_dev, void* stream) {
    if (!plan) return fr_fail(FRAMRIR_E_INVALID_ARG, "NULL plan");
    if (plan->header.multirate)
        return fr_fail(FRAMRIR_E_UNSUPPORTED, "multi-rate plan: use framrir_forward_multirate");
    if (plan->ws_bytes > static_cast<int64_t>(FRAMRIR_NOALLOC_SCRATCH_BYTES))
        return fr_fail(FRAMRIR_E_WORKSPACE,
                       "the plan needs %lld workspace bytes, the static scratch holds %lld: use framrir_forward "
                       "with a caller workspace, or split the batch",
                       static_cast<long long>(plan->ws_bytes),
                       static_cast<long long>(FRAMRIR_NOALLOC_SCRATCH_BYTES));
    void* ws = nullptr;
    int rc = current_scratch(&ws);
    if (rc) return rc;
    // every argument checked before anything is enqueued
    rc = check_render_args(plan, desc_dev, table_dev, mic_dev, src_dev, out_dev, ws,
                           static_cast<size_t>(FRAMRIR_NOALLOC_SCRATCH_BYTES), plan->ws_bytes, false);
    if (rc) return rc;
    // the persistent grid's counters start at zero: cleared by a kernel (not
    // a memset node, so that the call can be captured), every call
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(zero_counters_kernel, dim3(1), dim3(64), 0, st, static_cast<int*>(ws));
    if ((rc = check_launch("zero_counters_kernel"))) return rc;
    if ((rc = launch_prepare(plan, desc_dev, table_dev, mic_dev, src_dev, r_dev, ws, st, true))) return rc;
    return launch_render(plan, desc_dev, table_dev, mic_dev, src_dev, r_dev, out_dev, ws, st);
}

extern "C" int framrir_forward_early(const framrir_plan* plan, const void* desc_dev, double* table_dev,
                                     const double* mic_dev, const double* src_dev, const double* r_dev,
                                     float* out_dev, float* early_dev, int32_t* start_dev, void* ws_dev,
                                     size_t ws_bytes, void* stream) {
    if (plan && plan->header.multirate)
        return fr_fail(FRAMRIR_E_UNSUPPORTED, "multi-rate plan: the early windows are taken at the output rate");
    if (!early_dev) return fr_fail(FRAMRIR_E_INVALID_ARG, "early_dev is NULL (use framrir_forward)");
    int rc = check_render_args(plan, desc_dev, table_dev, mic_dev, src_dev, out_dev, ws_dev, ws_bytes,
                               plan ? plan->ws_bytes : 0, false);
    if (rc) return rc;
    if (!aligned(early_dev, 4)) return fr_fail(FRAMRIR_E_INVALID_ARG, "misaligned early_dev");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if ((rc = launch_prepare(plan, desc_dev, table_dev, mic_dev, src_dev, r_dev, ws_dev, st, true))) return rc;
    return launch_render(plan, desc_dev, table_dev, mic_dev, src_dev, r_dev, out_dev, ws_dev, st, early_dev,
                         start_dev);
}

namespace {

struct BwdArgs {
    const void* desc;
    const double* mic;
    const double* r;
    const float* grad_out;
    const double* sorted;
    const int* bucket_off;
    const int* row0_slot;
    int* room_done;
    float* partials;
    int* counters;
    float* grad_mic;
    float* grad_src;
    float* grad_r;
    int lds_words;
};

template <int NT, int WPE, bool DRAWS>
int launch_backward_kernel(dim3 grid, dim3 block, int lds, hipStream_t st, const BwdArgs& a) {
    if (int rc = allow_lds<backward_kernel<NT, WPE, DRAWS>>()) return rc;
    hipLaunchKernelGGL((backward_kernel<NT, WPE, DRAWS>), grid, block, lds, st, a.desc, a.mic, a.r, a.grad_out,
                       a.sorted, a.bucket_off, a.row0_slot, a.room_done, a.partials, a.counters, a.grad_mic,
                       a.grad_src, a.grad_r, a.lds_words);
    return FRAMRIR_OK;
}

int launch_backward(const framrir_plan* plan, const void* desc_dev, const double* mic_dev, const double* r_dev,
                    const float* grad_out_dev, float* grad_mic_dev, float* grad_src_dev, float* grad_r_dev,
                    void* ws_dev, size_t ws_bytes, hipStream_t st, bool draws) {
    if (plan && plan->header.multirate)
        return fr_fail(FRAMRIR_E_UNSUPPORTED, "multi-rate plan: use framrir_forward_multirate");
    if (!plan || !desc_dev || !mic_dev || !grad_out_dev || !ws_dev)
        return fr_fail(FRAMRIR_E_INVALID_ARG, "NULL argument");
    if (!aligned(desc_dev, 256) || !aligned(ws_dev, 256) || !aligned(grad_out_dev, 4))
        return fr_fail(FRAMRIR_E_INVALID_ARG, "misaligned buffer");
    if (static_cast<int64_t>(ws_bytes) < plan->ws_bwd_bytes)
        return fr_fail(FRAMRIR_E_WORKSPACE, "workspace %zu < %lld bytes", ws_bytes,
                       static_cast<long long>(plan->ws_bwd_bytes));
    const RenderWs w = render_ws(plan, ws_dev);
    float* partials = reinterpret_cast<float*>(static_cast<char*>(ws_dev) + plan->ws_part_off);
    // Through the draws the kernel runs at 4 waves per SIMD; there two
    // 512-thread workgroups per CU finish the persistent queue sooner than
    // one 1024-thread workgroup, so larger workgroups are capped at 512.
    const int nt = draws ? std::min(plan->launch.bwd_wg_threads, 512) : plan->launch.bwd_wg_threads;
    const int red_floats = (draws ? bwd_values<true>() : bwd_values<false>()) + 1;
    const int lds = std::max(plan->launch.lds_bytes, 4 * red_floats * nt);
    const dim3 grid(plan->bwd_grid), block(nt);
    // The adjoint through the draws holds 11 sums per thread and runs at 4
    // waves per SIMD whatever the launch asks (at 8 its registers spill).
    const int key = nt * 16 + (draws ? 4 : plan->launch.waves_per_simd);
    const BwdArgs args{desc_dev, mic_dev, r_dev, grad_out_dev, w.sorted, w.bucket_off, w.row0_slot, w.room_done,
                       partials, w.counters, grad_mic_dev, grad_src_dev, grad_r_dev, lds / 4};
    int rc = FRAMRIR_OK;
    switch (key) {
#define FR_CASE(NT, WPE)                                                                         \
    case NT * 16 + WPE:                                                                          \
        rc = (draws && WPE == 4) ? launch_backward_kernel<NT, 4, true>(grid, block, lds, st, args) \
                                 : launch_backward_kernel<NT, WPE, false>(grid, block, lds, st, args); \
        break;
        FR_KERNEL_SHAPES(FR_CASE)
#undef FR_CASE
        default:
            return fr_fail(FRAMRIR_E_UNSUPPORTED, "launch shape not compiled");
    }
    if (rc) return rc;
    return check_launch("backward_kernel");
}

}  // namespace

extern "C" int framrir_render_backward_prepared(const framrir_plan* plan, const void* desc_dev,
                                                const double* mic_dev, const double* r_dev,
                                                const float* grad_out_dev, float* grad_mic_dev, float* grad_src_dev,
                                                float* grad_r_dev, void* ws_dev, size_t ws_bytes, void* stream) {
    return launch_backward(plan, desc_dev, mic_dev, r_dev, grad_out_dev, grad_mic_dev, grad_src_dev, grad_r_dev,
                           ws_dev, ws_bytes, static_cast<hipStream_t>(stream), false);
}

extern "C" int framrir_render_backward(const framrir_plan* plan, const void* desc_dev, const double* table_dev,
                                       const double* mic_dev, const double* src_dev, const double* r_dev,
                                       const float* grad_out_dev, float* grad_mic_dev, float* grad_src_dev,
                                       float* grad_r_dev, void* ws_dev, size_t ws_bytes, void* stream) {
    if (plan && plan->header.multirate)
        return fr_fail(FRAMRIR_E_UNSUPPORTED, "multi-rate plan: use framrir_forward_multirate");
    int rc = check_render_args(plan, desc_dev, table_dev, mic_dev, src_dev, grad_out_dev, ws_dev, ws_bytes,
                               plan ? plan->ws_bwd_bytes : 0);
    if (rc) return rc;
    rc = launch_prepare(plan, desc_dev, const_cast<double*>(table_dev), mic_dev, src_dev, r_dev, ws_dev,
                        static_cast<hipStream_t>(stream), false);
    if (rc) return rc;
    return framrir_render_backward_prepared(plan, desc_dev, mic_dev, r_dev, grad_out_dev, grad_mic_dev,
                                            grad_src_dev, grad_r_dev, ws_dev, ws_bytes, stream);
}

extern "C" int framrir_render_backward_draws_prepared(const framrir_plan* plan, const void* desc_dev,
                                                      const double* mic_dev, const float* grad_out_dev,
                                                      float* grad_mic_dev, float* grad_src_dev, float* grad_r_dev,
                                                      void* ws_dev, size_t ws_bytes, void* stream) {
    return launch_backward(plan, desc_dev, mic_dev, nullptr, grad_out_dev, grad_mic_dev, grad_src_dev, grad_r_dev,
                           ws_dev, ws_bytes, static_cast<hipStream_t>(stream), true);
}

extern "C" int framrir_render_backward_draws(const framrir_plan* plan, const void* desc_dev,
                                             const double* table_dev, const double* mic_dev, const double* src_dev,
                                             const float* grad_out_dev, float* grad_mic_dev, float* grad_src_dev,
                                             float* grad_r_dev, void* ws_dev, size_t ws_bytes, void* stream) {
    if (plan && plan->header.multirate)
        return fr_fail(FRAMRIR_E_UNSUPPORTED, "multi-rate plan: use framrir_forward_multirate");
    int rc = check_render_args(plan, desc_dev, table_dev, mic_dev, src_dev, grad_out_dev, ws_dev, ws_bytes,
                               plan ? plan->ws_bwd_bytes : 0);
    if (rc) return rc;
    rc = launch_prepare(plan, desc_dev, const_cast<double*>(table_dev), mic_dev, src_dev, nullptr, ws_dev,
                        static_cast<hipStream_t>(stream), false);
    if (rc) return rc;
    return framrir_render_backward_draws_prepared(plan, desc_dev, mic_dev, grad_out_dev, grad_mic_dev, grad_src_dev,
                                                  grad_r_dev, ws_dev, ws_bytes, stream);
}

extern "C" int framrir_early(const framrir_plan* plan, const void* desc_dev, const double* mic_dev,
                             const double* src_dev, const float* out_dev, float* early_dev, int32_t* start_dev,
                             void* stream) {
    if (plan && plan->header.multirate)
        return fr_fail(FRAMRIR_E_UNSUPPORTED, "multi-rate plan: use framrir_forward_multirate");
    if (!plan || !desc_dev || !mic_dev || !src_dev || !out_dev || !early_dev)
        return fr_fail(FRAMRIR_E_INVALID_ARG, "NULL argument");
    if (!aligned(desc_dev, 256)) return fr_fail(FRAMRIR_E_INVALID_ARG, "misaligned descriptor");
    const DescHeader& H = plan->header;
    if (H.n_chan == 0) return FRAMRIR_OK;
    const unsigned gx = static_cast<unsigned>(std::min(8, (H.max_early + 255) / 256));
    const unsigned gy = static_cast<unsigned>(std::min(H.n_rooms, 65535));
    const unsigned gz = static_cast<unsigned>(std::min(H.max_room_chan, 1024));
    hipLaunchKernelGGL(early_kernel, dim3(gx, gy, gz), dim3(256), 0, static_cast<hipStream_t>(stream), desc_dev,
                       mic_dev, src_dev, out_dev, early_dev, start_dev);
    return check_launch("early_kernel");
}

extern "C" int framrir_multirate_filter(const framrir_plan* plan, const void* desc_dev, float* inter_dev,
                                        float* out_dev, void* ws_dev, size_t ws_bytes, void* stream);

extern "C" int framrir_forward_multirate(const framrir_plan* plan, const void* desc_dev, double* table_dev,
                                         const double* mic_dev, const double* src_dev, const double* r_dev,
                                         float* inter_dev, float* out_dev, void* ws_dev, size_t ws_bytes,
                                         void* stream) {
    int rc = check_render_args(plan, desc_dev, table_dev, mic_dev, src_dev, out_dev, ws_dev, ws_bytes,
                               plan ? plan->ws_mr_bytes : 0);
    if (rc) return rc;
    const DescHeader& H = plan->header;
    if (!H.multirate) return fr_fail(FRAMRIR_E_UNSUPPORTED, "not a multi-rate plan (FRAMRIR_FLAG_MULTIRATE)");
    if (!inter_dev || !aligned(inter_dev, 4)) return fr_fail(FRAMRIR_E_INVALID_ARG, "inter_dev NULL or misaligned");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if ((rc = launch_prepare(plan, desc_dev, table_dev, mic_dev, src_dev, r_dev, ws_dev, st, true))) return rc;
    if ((rc = launch_render(plan, desc_dev, table_dev, mic_dev, src_dev, r_dev, inter_dev, ws_dev, st))) return rc;
    return framrir_multirate_filter(plan, desc_dev, inter_dev, out_dev, ws_dev, ws_bytes, stream);
}

extern "C" int framrir_multirate_filter(const framrir_plan* plan, const void* desc_dev, float* inter_dev,
                                        float* out_dev, void* ws_dev, size_t ws_bytes, void* stream) {
    if (!plan || !desc_dev || !inter_dev || !out_dev || !ws_dev) return fr_fail(FRAMRIR_E_INVALID_ARG, "NULL argument");
    if (!aligned(desc_dev, 256) || !aligned(ws_dev, 256) || !aligned(inter_dev, 4) || !aligned(out_dev, 4))
        return fr_fail(FRAMRIR_E_INVALID_ARG, "misaligned buffer");
    const DescHeader& H = plan->header;
    if (!H.multirate) return fr_fail(FRAMRIR_E_UNSUPPORTED, "not a multi-rate plan (FRAMRIR_FLAG_MULTIRATE)");
    if (static_cast<int64_t>(ws_bytes) < plan->ws_mr_bytes)
        return fr_fail(FRAMRIR_E_WORKSPACE, "workspace %zu < %lld bytes", ws_bytes,
                       static_cast<long long>(plan->ws_mr_bytes));
    int rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    double* zend = reinterpret_cast<double*>(static_cast<char*>(ws_dev) + plan->ws_zend_off);
    double* init = reinterpret_cast<double*>(static_cast<char*>(ws_dev) + plan->ws_init_off);
    const unsigned gy = static_cast<unsigned>(std::min(H.n_rooms, 65535));
    const unsigned gz = static_cast<unsigned>(std::min(H.max_room_chan, 65535));
    double2* sub = reinterpret_cast<double2*>(static_cast<char*>(ws_dev) + plan->ws_sub_off);
    if (H.n_hp_tasks > 0) {   // persistent: about four workgroups per CU
        const unsigned g = static_cast<unsigned>(std::min(H.n_hp_tasks, kHpEndGrid));
        hipLaunchKernelGGL(hp_chunk_end_kernel, dim3(g), dim3(kHpEndThreads), 0, st, desc_dev, inter_dev, zend, sub);
        if ((rc = check_launch("hp_chunk_end_kernel"))) return rc;
    }
    hipLaunchKernelGGL(hp_carry_kernel, dim3(gy), dim3(64), 0, st, desc_dev, zend, init);
    if ((rc = check_launch("hp_carry_kernel"))) return rc;
    uint32_t* frag = reinterpret_cast<uint32_t*>(static_cast<char*>(ws_dev) + plan->ws_taps_off);
    hipLaunchKernelGGL(dec_frag_kernel, dim3(kMaxRl, kDmMaxSteps), dim3(64), 0, st, desc_dev, frag);
    if ((rc = check_launch("dec_frag_kernel"))) return rc;
    const int lds = 4 * dm_lds_words(H.max_rl);
    if (int rc2 = allow_lds<decimate_mfma_kernel, 4 * dm_lds_words(kMaxRl)>()) return rc2;
    hipLaunchKernelGGL(decimate_mfma_kernel, dim3(static_cast<unsigned>(std::min(H.max_out_tiles, 65535)), gy, gz),
                       dim3(kDmThreads), lds, st, desc_dev, inter_dev, init, sub, frag, out_dev);
    return check_launch("decimate_mfma_kernel");
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
