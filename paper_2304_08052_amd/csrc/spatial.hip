// gfx950 kernels of the spatialisation step of the on-the-fly training set-up
// (Sec. IV-A): each dry signal is convolved with its rendered multi-channel
// RIRs (overlap-save with a 32768-point real FFT held in one workgroup's LDS;
// an RIR longer than 16384 samples is cut into partitions of 16384 whose
// spectra multiply the signal's block spectra delayed by one block per
// partition, summed in partition order: uniformly partitioned overlap-save),
// the images' energies give the gains of the sampled SIR and SNR, and the
// scaled images are summed into the mixture.
//
//   fft_twiddle_kernel   exp(-2 pi i m / N) and exp(-2 pi i k / L), FP64 -> FP32
//   spectrum_kernel      real spectrum of an RIR channel or of a signal block
//   conv_block_kernel    product of the two spectra, inverse FFT, one output block
//   spatial_energy_kernel  per room: image energies (FP64, fixed order), in parts
//   spatial_gain_kernel  per room: the parts summed in order -> gains of the SIR and SNR
//   spatial_mix_kernel   scaled images (in place) and the mixture
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "../../include/framrir.h"
#include "framrir_internal.h"
#include "plan_internal.h"

namespace framrir {
namespace {

constexpr int kFftN = 16384;             // complex points: a real FFT of kFftL samples, two per point
constexpr int kFftL = 2 * kFftN;
constexpr int kFftThreads = 512;
constexpr int kBins = kFftN + 1;         // bins of the real spectrum
// The sequence lives in registers (32 points per thread); LDS carries the
// exchanges between passes, half of the sequence at a time, at padded
// positions i + i / 16 (the Stockham passes' strided writes then rarely meet
// in a bank), followed by two twiddle tables: w^m = T1[m / 64] T2[m mod 64],
// T1[h] = w^(64 h), T2[l] = w^l.  About 72 KB: two workgroups per CU, so
// that one's memory transfers overlap the other's passes.
constexpr int kHalfN = kFftN / 2;
constexpr int kHalfPadded = kHalfN + kHalfN / 16;
constexpr int kT1 = kFftN / 64, kT2 = 64;
constexpr int kFftLds = (kHalfPadded + kT1 + kT2) * 8;
__device__ __forceinline__ int pidx(int i) { return i + (i >> 4); }
constexpr int kSpatialSources = 3;       // two speakers and the noise (sources 0, 1, 2 of a room)

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(__builtin_fmaf(a.x, b.x, -a.y * b.y), __builtin_fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 conj2(float2 a) { return make_float2(a.x, -a.y); }

__global__ void fft_twiddle_kernel(float2* __restrict__ tw, float2* __restrict__ rt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double s, c;
    if (i < kFftN) {   // exp(-2 pi i m / N)
        sincospi(-2.0 * i / kFftN, &s, &c);
        tw[i] = make_float2(static_cast<float>(c), static_cast<float>(s));
    }
    if (i < kBins) {   // exp(-2 pi i k / L)
        sincospi(-2.0 * i / kFftL, &s, &c);
        rt[i] = make_float2(static_cast<float>(c), static_cast<float>(s));
    }
}

// 4-point forward DFT: X_q = sum_r v_r (-i)^(r q).
__device__ __forceinline__ void dft4(float2& a, float2& b, float2& c, float2& d) {
    const float2 s02 = cadd(a, c), d02 = csub(a, c), s13 = cadd(b, d), d13 = csub(b, d);
    const float2 jd13 = make_float2(d13.y, -d13.x);   // -i (v1 - v3)
    a = cadd(s02, s13);
    b = cadd(d02, jd13);
    c = csub(s02, s13);
    d = csub(d02, jd13);
}

// 16-point forward DFT in registers, natural order in and out: with n = n2 +
// 4 n1 and k = k1 + 4 k2, X_k = sum_n2 w16^(n2 k1) w4^(n2 k2) sum_n1 x_(n2 +
// 4 n1) w4^(n1 k1): 4-point DFTs over n1, the twiddles w16^(n2 k1), 4-point
// DFTs over n2.
__device__ __forceinline__ void dft16(float2 (&v)[16]) {
    constexpr float c1 = 0.92387953251128674f, s1 = 0.38268343236508978f, h = 0.70710678118654752f;
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4(v[n2], v[n2 + 4], v[n2 + 8], v[n2 + 12]);
    // v[n2 + 4 k1] now holds Y[n2][k1]; multiply by w16^(n2 k1)
    v[5] = cmul(v[5], make_float2(c1, -s1));     // w16^1
    v[6] = cmul(v[6], make_float2(h, -h));       // w16^2
    v[7] = cmul(v[7], make_float2(s1, -c1));     // w16^3
    v[9] = cmul(v[9], make_float2(h, -h));       // w16^2
    v[10] = make_float2(v[10].y, -v[10].x);      // w16^4 = -i
    v[11] = cmul(v[11], make_float2(-h, -h));    // w16^6
    v[13] = cmul(v[13], make_float2(s1, -c1));   // w16^3
    v[14] = cmul(v[14], make_float2(-h, -h));    // w16^6
    v[15] = cmul(v[15], make_float2(-c1, s1));   // w16^9
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) dft4(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
    // v[4 k1 + k2] holds X[k1 + 4 k2]: transpose the 4 x 4 index
    float2 t;
    t = v[1], v[1] = v[4], v[4] = t;
    t = v[2], v[2] = v[8], v[8] = t;
    t = v[3], v[3] = v[12], v[12] = t;
    t = v[6], v[6] = v[9], v[9] = t;
    t = v[7], v[7] = v[13], v[13] = t;
    t = v[11], v[11] = v[14], v[14] = t;
}

// w^m = T1[m / 64] T2[m mod 64], w = exp(-2 pi i / kFftN), m < kFftN.
__device__ __forceinline__ float2 twiddle(const float2* __restrict__ t1, const float2* __restrict__ t2, int m) {
    return cmul(t1[m >> 6], t2[m & 63]);
}

// The 15 twiddles w^(r step) of a radix-16 butterfly, r = 1..15, as products
// of w^step and w^(4 step) (at most three roundings deep).
__device__ __forceinline__ void twiddle16(const float2* __restrict__ t1, const float2* __restrict__ t2, int step,
                                          float2 (&v)[16]) {
    float2 w[16];
    w[1] = twiddle(t1, t2, step);
    w[4] = twiddle(t1, t2, 4 * step);
    w[2] = cmul(w[1], w[1]);
    w[3] = cmul(w[1], w[2]);
    w[5] = cmul(w[4], w[1]);
    w[6] = cmul(w[4], w[2]);
    w[7] = cmul(w[4], w[3]);
    w[8] = cmul(w[4], w[4]);
    w[9] = cmul(w[8], w[1]);
    w[10] = cmul(w[8], w[2]);
    w[11] = cmul(w[8], w[3]);
    w[12] = cmul(w[8], w[4]);
    w[13] = cmul(w[12], w[1]);
    w[14] = cmul(w[12], w[2]);
    w[15] = cmul(w[12], w[3]);
#pragma unroll
    for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], w[r]);
}

// Forward DFT of kFftN points, Stockham passes: three of radix 16 (stride
// Ns = 1, 16, 256), then one of radix 4 (Ns = 4096).  Butterfly j of a
// radix-R pass takes x[j + r N/R] (r = 0..R-1), multiplied by w^(r k N / (R
// Ns)) with k = j mod Ns, and its R-point DFT goes to (j / Ns) R Ns + k + q
// Ns.  Thread t runs butterflies t and t + 512 of each radix-16 pass (their
// outputs fill the lower and the upper half of the sequence) and t + 512 i,
// i = 0..7, of the radix-4 pass.  Between passes the outputs go through the
// LDS buffer buf one half at a time: the lower half is written, every thread
// reads the next pass's inputs that lie there, then the same for the upper
// half.  input(p) gives the sequence at position p; on return y[i][q] holds
// the DFT at t + 512 i + 4096 q.  v[b][r]: the sequence at t + 512 b + 1024
// r (overwritten).  t1, t2: the twiddle tables in LDS, loaded and
// synchronised by the caller.
__device__ __forceinline__ void fft16k(float2* __restrict__ buf, const float2* __restrict__ t1,
                                       const float2* __restrict__ t2, float2 (&v)[2][16], float2 (&y)[8][4]) {
    static_assert(kFftN == 16 * 16 * 16 * 4 && kFftN / 32 == kFftThreads, "pass plan of the 16384-point FFT");
    const int t = threadIdx.x;
#pragma unroll
    for (int shift = 0; shift < 12; shift += 4) {
        const int Ns = 1 << shift;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            if (shift > 0) twiddle16(t1, t2, ((t + 512 * b) & (Ns - 1)) << (10 - shift), v[b]);
            dft16(v[b]);
        }
        // butterfly b's outputs lie in half b; the next pass's inputs are
        // (radix 16) positions t + 512 b + 1024 r, in half r / 8, or
        // (radix 4) positions t + 512 i + 4096 r, in half r / 2
        float2 u[32];
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const int j = t + 512 * half;
            const int base = ((j >> shift) << (shift + 4)) + (j & (Ns - 1)) - kHalfN * half;
#pragma unroll
            for (int q = 0; q < 16; ++q) buf[pidx(base + q * Ns)] = v[half][q];
            __syncthreads();
            if (shift < 8) {
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int r = 8 * half; r < 8 * half + 8; ++r)
                        u[16 * b + r] = buf[pidx(t + 512 * b + 1024 * r - kHalfN * half)];
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i)
#pragma unroll
                    for (int r = 2 * half; r < 2 * half + 2; ++r)
                        u[4 * i + r] = buf[pidx(t + 512 * i + 4096 * r - kHalfN * half)];
            }
            __syncthreads();
        }
        if (shift < 8) {
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 16; ++r) v[b][r] = u[16 * b + r];
        } else {
            // radix 4, Ns = 4096: butterfly j = t + 512 i < 4096, so k = j
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int j = t + 512 * i;
                const float2 w1 = twiddle(t1, t2, j), w2 = cmul(w1, w1), w3 = cmul(w2, w1);
                y[i][0] = u[4 * i];
                y[i][1] = cmul(u[4 * i + 1], w1);
                y[i][2] = cmul(u[4 * i + 2], w2);
                y[i][3] = cmul(u[4 * i + 3], w3);
                dft4(y[i][0], y[i][1], y[i][2], y[i][3]);
            }
        }
    }
}

// The twiddle tables into LDS (after the exchange buffer); the caller
// synchronises before the first pass that reads them.
__device__ __forceinline__ void load_twiddles(float2* buf, const float2* __restrict__ tw) {
    float2* t1 = buf + kHalfPadded;
    for (int i = threadIdx.x; i < kT1 + kT2; i += kFftThreads) t1[i] = i < kT1 ? tw[64 * i] : tw[i - kT1];
}

// Room of a channel (binary search on the rooms' first channels).
__device__ __forceinline__ int room_of_chan(const void* desc, int c) {
    const DescHeader* H = hdr(desc);
    const RoomDesc* R = rooms(desc);
    int lo = 0, hi = H->n_rooms - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (R[mid].chan0 <= c) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Bin k of the real spectrum from zk = Z[k] and zc = conj(Z[N - k]) (Z[N] =
// Z[0]): X[k] = (zk + zc) / 2 - (i / 2) e^(-2 pi i k / L) (zk - zc).
__device__ __forceinline__ float2 real_bin(float2 zk, float2 zc, float2 rk) {
    const float2 e = make_float2(0.5f * (zk.x + zc.x), 0.5f * (zk.y + zc.y));
    const float2 d = cmul(rk, make_float2(0.5f * (zk.x - zc.x), 0.5f * (zk.y - zc.y)));
    return make_float2(e.x + d.y, e.y - d.x);   // e - i d
}

// Spectrum of a real segment of kFftL samples: packed as z[n] = s[2n] + i
// s[2n+1] and transformed; bins k and N - k both need Z[k] and Z[N - k],
// which thread pairs (t, 512 - t) exchange through the LDS buffer.  Jobs: one
// per (RIR channel, partition p) (RIR samples p Pl .. p Pl + Pl - 1 at the
// start of the segment, zeros after them; Pl the partition length), then one
// per (source, block j) (signal samples j B - (Pl - 1) + n, zeros outside
// [0, N_s)).
__global__ void __launch_bounds__(kFftThreads) __attribute__((amdgpu_waves_per_eu(4)))
spectrum_kernel(const void* __restrict__ desc, const float* __restrict__ rir, const float* __restrict__ sig,
                const float2* __restrict__ tw, const float2* __restrict__ rt, float2* __restrict__ hspec,
                float2* __restrict__ xspec, int n_chan, int n_part, int n_blk, int adv, int pl, int n_samples) {
    extern __shared__ float2 buf[];
    const int job = blockIdx.x;
    const float* seg;
    int64_t first;          // sample index of segment position 0
    int len;                // valid samples of the source sequence
    float2* dst;
    if (job < n_chan * n_part) {
        const int c = job / n_part, p = job - c * n_part;
        const int b = room_of_chan(desc, c);
        const RoomDesc& R = rooms(desc)[b];
        seg = rir + R.out2_off + static_cast<int64_t>(c - R.chan0) * R.T_out + static_cast<int64_t>(p) * pl;
        first = 0;
        len = min(pl, R.T_out - p * pl);   // may be <= 0: a zero spectrum
        dst = hspec + static_cast<int64_t>(job) * kBins;
    } else {
        const int q = job - n_chan * n_part, s = q / n_blk, j = q % n_blk;
        seg = sig + static_cast<int64_t>(s) * n_samples;
        first = static_cast<int64_t>(j) * adv - (pl - 1);
        len = n_samples;
        dst = xspec + static_cast<int64_t>(q) * kBins;
    }
    load_twiddles(buf, tw);
    const int t = threadIdx.x;
    float2 v[2][16];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t i0 = first + 2 * (t + 512 * b + 1024 * r), i1 = i0 + 1;
            v[b][r] = make_float2(i0 >= 0 && i0 < len ? seg[i0] : 0.0f, i1 >= 0 && i1 < len ? seg[i1] : 0.0f);
        }
    __syncthreads();
    const float2* t1 = buf + kHalfPadded;
    float2 y[8][4];
    fft16k(buf, t1, t1 + kT1, v, y);
    // y[i][q] is Z at p = t + 512 i + 4096 q; for t >= 1 the partner N - p is
    // (512 - t, 7 - i, 3 - q): the q >= 2 values go to the LDS buffer (slot
    // (2 i + q - 2) 512 + t) and thread t forms bins p and N - p for its q < 2
    // positions from its own value and its partner's.  Thread 0 does the
    // same with partners among its own values, (N - p) mod N = (8 - i, 3 - q)
    // or, for i = 0, (0, -q mod 4), which also gives bin N from p = 0; bin
    // N/2 (its position (0, 2)) it forms alone.
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int q = 2; q < 4; ++q) buf[(2 * i + q - 2) * kFftThreads + t] = y[i][q];
    __syncthreads();
    const int tp = (kFftThreads - t) & (kFftThreads - 1);   // partner thread (thread 0: unused slot)
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int p = t + 512 * i + 4096 * q;
            const float2 own = i == 0 ? y[0][(4 - q) & 3] : y[8 - i][3 - q];
            const float2 zp = t == 0 ? own : buf[(2 * (7 - i) + 1 - q) * kFftThreads + tp];
            dst[p] = real_bin(y[i][q], conj2(zp), rt[p]);
            dst[kFftN - p] = real_bin(zp, conj2(y[i][q]), rt[kFftN - p]);
        }
    if (t == 0) dst[kHalfN] = real_bin(y[0][2], conj2(y[0][2]), rt[kHalfN]);
}

// One output block of one channel: P = sum_p X_(j-p) H_p over the RIR's
// partitions (block spectra of the signal delayed by p blocks; terms added in
// partition order), then the inverse real FFT by the forward one: Z[k] = E[k]
// + i O[k], E = (P[k] + P*[N-k]) / 2, O = (P[k] - P*[N-k]) e^(2 pi i k / L) /
// 2, z = conj(DFT(conj(Z))) / N, samples 2n and 2n+1 = Re, Im z[n].  Samples
// Pl - 1 .. Pl - 2 + B of the block are the outputs j B .. j B + B - 1
// (overlap-save; B = L - Pl + 1 for one partition, B = Pl for several).
// Each thread forms P at its own input
// positions k and takes P[N - k] from the thread that formed it, through the
// LDS buffer half by half (k = 0 pairs with the Nyquist bin P[N], k = N/2
// with itself); e^(2 pi i k / L) comes from the LDS twiddle tables.
template <bool PARTS>   // false: one partition (the products need no sum)
__global__ void __launch_bounds__(kFftThreads) __attribute__((amdgpu_waves_per_eu(4)))
conv_block_kernel(const void* __restrict__ desc, const float2* __restrict__ tw, const float2* __restrict__ hspec,
                  const float2* __restrict__ xspec, float* __restrict__ images, int n_part, int n_blk, int adv,
                  int pl, int n_samples) {
    extern __shared__ float2 buf[];
    const int c = blockIdx.x / n_blk, j = blockIdx.x % n_blk;
    const int b = room_of_chan(desc, c);
    const RoomDesc& R = rooms(desc)[b];
    const int s = R.src0 + (c - R.chan0) / R.n_mic;
    const float2* H = hspec + static_cast<int64_t>(c) * n_part * kBins;        // partition p at + p kBins
    const float2* X = xspec + (static_cast<int64_t>(s) * n_blk + j) * kBins;   // block j - p at - p kBins
    const int n_terms = min(n_part, j + 1);   // blocks before the signal start are zero
    auto product = [&](int k) {               // sum_p X_(j-p)[k] H_p[k], p ascending
        float2 acc = cmul(X[k], H[k]);
        if constexpr (PARTS)
        for (int p = 1; p < n_terms; ++p) {
            const float2 v = cmul(X[k - static_cast<int64_t>(p) * kBins], H[k + static_cast<int64_t>(p) * kBins]);
            acc = make_float2(acc.x + v.x, acc.y + v.y);
        }
        return acc;
    };
    load_twiddles(buf, tw);
    const int t = threadIdx.x;
    // Z[k] needs P[k] = X[k] H[k] and P[N - k].  The thread's positions are
    // k = t + 512 b + 1024 r; for t >= 1 the partner of (t, b = 0, r) is (512
    // - t, b = 1, 15 - r), so thread t forms both Z of each of its b = 0
    // pairs: the b = 1 products go to the LDS buffer (slot r 512 + t), the
    // thread reads its partner's product there and puts the partner's Z in
    // its place.  Thread 0's pairs are among its own positions (0 with the
    // Nyquist bin P[N], N/2 with itself).  r_(N - k) = -conj(r_k).
    const float2* t1 = buf + kHalfPadded;
    auto rt_of = [&](int k) {   // e^(-2 pi i k / L)
        const float2 wl = make_float2(0.99999998161642933f, -1.9174759731070331e-4f);   // e^(-pi i / N)
        const float2 tk = twiddle(t1, t1 + kT1, k >> 1);
        return (k & 1) ? cmul(tk, wl) : tk;
    };
    auto zform = [](float2 pk, float2 pnk, float2 rk) {   // Z[k] from P[k], P[N - k], r_k
        const float2 pc = conj2(pnk);
        const float2 e = make_float2(0.5f * (pk.x + pc.x), 0.5f * (pk.y + pc.y));
        const float2 o = cmul(conj2(rk), make_float2(0.5f * (pk.x - pc.x), 0.5f * (pk.y - pc.y)));
        return make_float2(e.x - o.y, -(e.y + o.x));   // conj(e + i o)
    };
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int k = t + 512 + 1024 * r;
        buf[r * kFftThreads + t] = product(k);
    }
    float2 v[2][16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int k = t + 1024 * r;
        v[0][r] = product(k);
    }
    __syncthreads();
    if (t != 0) {
        const int tp = kFftThreads - t;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            float2* slot = buf + (15 - r) * kFftThreads + tp;
            const float2 p = *slot;
            const float2 rk = rt_of(t + 1024 * r);
            *slot = zform(p, v[0][r], make_float2(-rk.x, rk.y));
            v[0][r] = zform(v[0][r], p, rk);
        }
    } else {
        const float2 pn = product(kFftN);
#pragma unroll
        for (int r = 0; r < 8; ++r) {   // b = 1: (512 + 1024 r) with (512 + 1024 (15 - r))
            const float2 a1 = buf[r * kFftThreads], b1 = buf[(15 - r) * kFftThreads];
            buf[r * kFftThreads] = zform(a1, b1, rt_of(512 + 1024 * r));
            buf[(15 - r) * kFftThreads] = zform(b1, a1, rt_of(512 + 1024 * (15 - r)));
        }
#pragma unroll
        for (int r = 1; r < 8; ++r) {   // b = 0: 1024 r with 1024 (16 - r)
            const float2 a0 = v[0][r], b0 = v[0][16 - r];
            v[0][r] = zform(a0, b0, rt_of(1024 * r));
            v[0][16 - r] = zform(b0, a0, rt_of(1024 * (16 - r)));
        }
        v[0][0] = zform(v[0][0], pn, rt_of(0));
        v[0][8] = zform(v[0][8], v[0][8], rt_of(kHalfN));
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) v[1][r] = buf[r * kFftThreads + t];
    __syncthreads();   // the transform reuses the buffer
    float2 y[8][4];
    fft16k(buf, t1, t1 + kT1, v, y);
    constexpr float inv_n = 1.0f / kFftN;
    float* out = images + static_cast<int64_t>(c) * n_samples;
    const int o0 = j * adv - (pl - 1);   // output index of segment sample 0 (n_samples < 2^31)
    const int lo = pl - 1, hi = pl - 1 + adv;   // the block's outputs (each written by one block only)
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int n2 = 2 * (static_cast<int>(threadIdx.x) + 512 * i + 4096 * q);
            if (n2 >= lo && n2 < hi && o0 + n2 < n_samples) out[o0 + n2] = y[i][q].x * inv_n;
            if (n2 + 1 >= lo && n2 + 1 < hi && o0 + n2 + 1 < n_samples) out[o0 + n2 + 1] = -y[i][q].y * inv_n;
        }
}

// Per room: E1, E2, E12 = sum y0 y1 and En over all microphones and samples,
// split over kEnergyParts workgroups (blocks (part, room)), each thread
// summing a fixed set of samples in FP64, then a fixed reduction tree; one
// set of partial sums per workgroup.
constexpr int kEnergyParts = 64;
constexpr int kEnergyThreads = 256;
__global__ void __launch_bounds__(kEnergyThreads) spatial_energy_kernel(const void* __restrict__ desc,
                                                                        const float* __restrict__ images,
                                                                        double* __restrict__ partials,
                                                                        int n_samples) {
    __shared__ double red[4][kEnergyThreads];
    const int part = blockIdx.x, b = blockIdx.y;
    const RoomDesc& R = rooms(desc)[b];
    const int tid = threadIdx.x;
    const int64_t per = static_cast<int64_t>(R.n_mic) * n_samples;   // samples of one source's image
    const float* y0 = images + static_cast<int64_t>(R.chan0) * n_samples;
    const float* y1 = y0 + per;
    const float* y2 = y1 + per;
    double e1 = 0.0, e2 = 0.0, e12 = 0.0, en = 0.0;
    for (int64_t i = static_cast<int64_t>(part) * kEnergyThreads + tid; i < per;
         i += static_cast<int64_t>(kEnergyParts) * kEnergyThreads) {
        const double a0 = y0[i], a1 = y1[i], a2 = y2[i];
        e1 += a0 * a0;
        e2 += a1 * a1;
        e12 += a0 * a1;
        en += a2 * a2;
    }
    red[0][tid] = e1;
    red[1][tid] = e2;
    red[2][tid] = e12;
    red[3][tid] = en;
    __syncthreads();
    for (int w = kEnergyThreads / 2; w > 0; w >>= 1) {
        if (tid < w)
            for (int q = 0; q < 4; ++q) red[q][tid] += red[q][tid + w];
        __syncthreads();
    }
    if (tid < 4) partials[(static_cast<int64_t>(b) * kEnergyParts + part) * 4 + tid] = red[tid][0];
}

// Per room (one wave): the partial energies summed by a fixed tree (lane l
// takes parts l, l + 64, ..., then a butterfly over the lanes), then the gains
// (1, g2, gn) of the room's SIR and SNR (a silent source gets gain 0).
__global__ void __launch_bounds__(64) spatial_gain_kernel(const void* __restrict__ desc,
                                                          const double* __restrict__ partials,
                                                          const float* __restrict__ sir_db,
                                                          const float* __restrict__ snr_db, float* __restrict__ gains) {
    const int b = blockIdx.x, lane = threadIdx.x;
    const RoomDesc& R = rooms(desc)[b];
    double e[4] = {0.0, 0.0, 0.0, 0.0};
    const double* pb = partials + static_cast<int64_t>(b) * kEnergyParts * 4;
    for (int p = lane; p < kEnergyParts; p += 64)
        for (int q = 0; q < 4; ++q) e[q] += pb[4 * p + q];
    for (int off = 32; off > 0; off >>= 1)
        for (int q = 0; q < 4; ++q) e[q] += __shfl_xor(e[q], off);
    if (lane != 0) return;
    const double e1 = e[0], e2 = e[1], e12 = e[2], en = e[3];
    const double g2 = e2 > 0.0 ? sqrt(e1 / (e2 * exp10(static_cast<double>(sir_db[b]) / 10.0))) : 0.0;
    const double esp = e1 + 2.0 * g2 * e12 + g2 * g2 * e2;
    const double gn = en > 0.0 ? sqrt(esp / (en * exp10(static_cast<double>(snr_db[b]) / 10.0))) : 0.0;
    gains[R.src0] = 1.0f;
    gains[R.src0 + 1] = static_cast<float>(g2);
    gains[R.src0 + 2] = static_cast<float>(gn);
}

// Scaled images (in place) and the mixture; blocks (chunk, room).
__global__ void spatial_mix_kernel(const void* __restrict__ desc, float* __restrict__ images,
                                   const float* __restrict__ gains, float* __restrict__ mix, int n_samples) {
    const int b = blockIdx.y;
    const RoomDesc& R = rooms(desc)[b];
    const int64_t per = static_cast<int64_t>(R.n_mic) * n_samples;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= per) return;
    float* y = images + static_cast<int64_t>(R.chan0) * n_samples;
    const float* g = gains + R.src0;
    const float v0 = y[i] * g[0], v1 = y[per + i] * g[1], v2 = y[2 * per + i] * g[2];
    y[i] = v0;
    y[per + i] = v1;
    y[2 * per + i] = v2;
    mix[static_cast<int64_t>(R.mic0) * n_samples + i] = (v0 + v1) + v2;
}

// RIRs up to kFftN samples: one partition of the RIR's length Tm, blocks of
// B = L - Tm + 1 outputs.  Longer ones (at most kMaxPart partitions): Pl =
// kFftN, B = Pl.
constexpr int kMaxPart = 16;

struct SpatialLayout {
    int tm, pl, n_part, adv, n_blk;
    int64_t tw_off, rt_off, h_off, x_off, e_off, bytes;
};

int spatial_layout(const framrir_plan* plan, int32_t n_samples, SpatialLayout& L) {
    if (!plan) return fr_fail(FRAMRIR_E_INVALID_ARG, "plan is NULL");
    if (n_samples < 1) return fr_fail(FRAMRIR_E_INVALID_ARG, "n_samples = %d must be >= 1", n_samples);
    int tm = 1;
    for (const RoomDesc& R : plan->rooms) {
        if (R.n_src != kSpatialSources)
            return fr_fail(FRAMRIR_E_INVALID_ARG, "spatialisation needs 3 sources per room (two speakers, the noise)");
        tm = std::max(tm, static_cast<int>(R.T_out));
    }
    if (tm > kMaxPart * kFftN)
        return fr_fail(FRAMRIR_E_UNSUPPORTED, "RIRs of %d samples: the spatialisation takes at most %d", tm,
                       kMaxPart * kFftN);
    auto align = [](int64_t v) { return (v + 255) & ~int64_t(255); };
    L.tm = tm;
    L.n_part = (tm + kFftN - 1) / kFftN;
    L.pl = L.n_part == 1 ? tm : kFftN;
    L.adv = kFftL - L.pl + (L.n_part == 1 ? 1 : 0);
    L.n_blk = static_cast<int>((static_cast<int64_t>(n_samples) + L.adv - 1) / L.adv);
    L.tw_off = 0;
    L.rt_off = align(L.tw_off + 8 * static_cast<int64_t>(kFftN));
    L.h_off = align(L.rt_off + 8 * static_cast<int64_t>(kBins));
    L.x_off = align(L.h_off + 8 * static_cast<int64_t>(kBins) * plan->header.n_chan * L.n_part);
    L.e_off = align(L.x_off + 8 * static_cast<int64_t>(kBins) * plan->header.n_src * L.n_blk);
    L.bytes = align(L.e_off + 8 * 4 * static_cast<int64_t>(kEnergyParts) * plan->header.n_rooms);
    return FRAMRIR_OK;
}

int allow_fft_lds() {
    static int status = [] {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(spectrum_kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, kFftLds);
        if (e == hipSuccess)
            e = hipFuncSetAttribute(reinterpret_cast<const void*>(conv_block_kernel<false>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, kFftLds);
        if (e == hipSuccess)
            e = hipFuncSetAttribute(reinterpret_cast<const void*>(conv_block_kernel<true>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, kFftLds);
        return e == hipSuccess ? 0 : static_cast<int>(e);
    }();
    if (status != 0)
        return fr_fail(FRAMRIR_E_DEVICE, "hipFuncSetAttribute: %s", hipGetErrorString(static_cast<hipError_t>(status)));
    return FRAMRIR_OK;
}

int check(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fr_fail(FRAMRIR_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
    return FRAMRIR_OK;
}

}  // namespace
}  // namespace framrir

using namespace framrir;

extern "C" int framrir_spatial_workspace(const framrir_plan* plan, int32_t n_samples, size_t* ws_bytes) {
    if (!ws_bytes) return fr_fail(FRAMRIR_E_INVALID_ARG, "ws_bytes is NULL");
    SpatialLayout L;
    if (int rc = spatial_layout(plan, n_samples, L)) return rc;
    *ws_bytes = static_cast<size_t>(L.bytes);
    return FRAMRIR_OK;
}

extern "C" int framrir_spatialize(const framrir_plan* plan, const void* desc_dev, const float* rir_dev,
                                  const float* sig_dev, const float* sir_db_dev, const float* snr_db_dev,
                                  int32_t n_samples, float* images_dev, float* mix_dev, float* gains_dev,
                                  void* ws_dev, size_t ws_bytes, void* stream) {
    SpatialLayout L;
    if (int rc = spatial_layout(plan, n_samples, L)) return rc;
    if (!desc_dev || !rir_dev || !sig_dev || !sir_db_dev || !snr_db_dev || !images_dev || !mix_dev || !gains_dev ||
        !ws_dev)
        return fr_fail(FRAMRIR_E_INVALID_ARG, "NULL argument");
    if (reinterpret_cast<uintptr_t>(ws_dev) % 256 != 0 || reinterpret_cast<uintptr_t>(desc_dev) % 256 != 0)
        return fr_fail(FRAMRIR_E_INVALID_ARG, "misaligned buffer");
    if (static_cast<int64_t>(ws_bytes) < L.bytes)
        return fr_fail(FRAMRIR_E_WORKSPACE, "workspace %zu < %lld bytes", ws_bytes, static_cast<long long>(L.bytes));
    if (int rc = allow_fft_lds()) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(ws_dev);
    float2* tw = reinterpret_cast<float2*>(w + L.tw_off);
    float2* rt = reinterpret_cast<float2*>(w + L.rt_off);
    float2* hspec = reinterpret_cast<float2*>(w + L.h_off);
    float2* xspec = reinterpret_cast<float2*>(w + L.x_off);
    const int n_chan = plan->header.n_chan, n_src = plan->header.n_src, n_rooms = plan->header.n_rooms;
    hipLaunchKernelGGL(fft_twiddle_kernel, dim3((kBins + 255) / 256), dim3(256), 0, st, tw, rt);
    if (int rc = check("fft_twiddle_kernel")) return rc;
    hipLaunchKernelGGL(spectrum_kernel, dim3(n_chan * L.n_part + n_src * L.n_blk), dim3(kFftThreads), kFftLds, st,
                       desc_dev, rir_dev, sig_dev, tw, rt, hspec, xspec, n_chan, L.n_part, L.n_blk, L.adv, L.pl,
                       n_samples);
    if (int rc = check("spectrum_kernel")) return rc;
    if (L.n_part == 1)
        hipLaunchKernelGGL(conv_block_kernel<false>, dim3(n_chan * L.n_blk), dim3(kFftThreads), kFftLds, st, desc_dev,
                           tw, hspec, xspec, images_dev, L.n_part, L.n_blk, L.adv, L.pl, n_samples);
    else
        hipLaunchKernelGGL(conv_block_kernel<true>, dim3(n_chan * L.n_blk), dim3(kFftThreads), kFftLds, st, desc_dev,
                           tw, hspec, xspec, images_dev, L.n_part, L.n_blk, L.adv, L.pl, n_samples);
    if (int rc = check("conv_block_kernel")) return rc;
    double* partials = reinterpret_cast<double*>(w + L.e_off);
    hipLaunchKernelGGL(spatial_energy_kernel, dim3(kEnergyParts, n_rooms), dim3(kEnergyThreads), 0, st, desc_dev,
                       images_dev, partials, n_samples);
    if (int rc = check("spatial_energy_kernel")) return rc;
    hipLaunchKernelGGL(spatial_gain_kernel, dim3(n_rooms), dim3(64), 0, st, desc_dev, partials, sir_db_dev,
                       snr_db_dev, gains_dev);
    if (int rc = check("spatial_gain_kernel")) return rc;
    int max_per = 0;
    for (const RoomDesc& R : plan->rooms) max_per = std::max(max_per, R.n_mic);
    const int64_t per = static_cast<int64_t>(max_per) * n_samples;
    hipLaunchKernelGGL(spatial_mix_kernel, dim3(static_cast<unsigned>((per + 255) / 256), n_rooms), dim3(256), 0, st,
                       desc_dev, images_dev, gains_dev, mix_dev, n_samples);
    return check("spatial_mix_kernel");
}
