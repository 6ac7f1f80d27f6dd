// Internal layout of the FRAM-RIR device descriptor blob and the numeric
// helpers shared by the host planner and the gfx950 kernels of this library.
//
// Everything in the blob is 8-byte aligned plain data.  The host planner
// (plan.cpp) writes it; the kernels (kernels.hip) read it.
#pragma once

#include <math.h>
#include <stdint.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define FR_HD __host__ __device__ inline
#else
#define FR_HD inline
#endif

namespace framrir {

constexpr int kTaps = 81;
constexpr int kHalf = 40;          // taps are k - 40 .. k + 40 around k = floor(t + 1/2)
constexpr int kHalo = 80;          // LDS guard samples on each side of a time tile
constexpr int kMaxMicGroup = 16;   // microphones per work item
constexpr int kBuckets = 1024;     // delay buckets of the per-source row order
constexpr int kLdsBanks = 32;      // LDS banks of gfx950 (4 bytes each)
constexpr int kPool = 128;         // render: pairs a wave ranks by bank per round (two per lane)
// Static LDS of the render kernel for a workgroup of nt threads, bounded from
// above: per wave the staged pool (3 words per pair) and the bank counts,
// plus the microphone group and the item slot.
constexpr int render_static_lds(int nt) { return 512 + (nt / 64) * (3 * kPool + kLdsBanks) * 4; }
// Backward partials per item: dL/dmic per microphone of the group (3 each),
// then dL/dsrc through the direct path (3), dL/dr, and for the gradient
// through the draws the sum of dL/dpos over the item's images (3) and dL/dd0.
constexpr int kPartialStride = 3 * kMaxMicGroup + 8;
constexpr int kPartSrc = 3 * kMaxMicGroup, kPartR = kPartSrc + 3, kPartPos = kPartR + 1, kPartD0 = kPartPos + 3;

enum TauCode : int32_t { kTauQuarter = 0, kTauHalf = 1, kTauOne = 2 };

struct DescHeader {
    int32_t n_rooms, n_src, n_mic, n_items;
    int64_t n_img, out_floats;
    int64_t room_bytes, src_bytes, item_bytes, room_items_bytes;   // byte offsets in the blob
    double alpha, beta, a, b;
    double a3, b3;             // alpha^3 and beta^3, each product rounded separately
    double beta_minus_alpha, b_minus_a;
    int32_t tau_code;
    int32_t max_img;           // largest I + 1 of the batch
    int32_t max_T;
    int32_t n_chan;            // sum over rooms of n_src * n_mic
    int64_t early_floats;      // floats of the packed early-reverberation windows
    int32_t max_early;         // longest early window (samples)
    int32_t max_room_chan;     // largest n_src * n_mic of a room
    // multi-rate plans (Sec. II): the render works at r_l fs into an
    // intermediate buffer of mr_floats; out_floats is the output at fs
    int32_t multirate;
    int32_t max_chunks;        // high-pass chunks per channel, at most
    int64_t mr_floats;
    int64_t n_chunks;          // high-pass chunks of the batch
    int32_t max_out_tiles;     // decimation tiles per channel, at most
    int32_t max_rl;
    int64_t src_order_bytes;   // byte offset of int32[n_src]: the sources by row count, largest first
    int64_t hp_task_bytes;     // byte offset of HpTask[n_hp_tasks] (multi-rate plans)
    int32_t n_hp_tasks;        // high-pass blocks of kHpEndChunks chunks over all channels
    int32_t pad_hp;
};

// One block of the high-pass state pass: kHpEndChunks consecutive chunks of
// one channel (room b, channel chan = s n_mic + m of the room, first chunk
// kHpEndChunks blk).
struct HpTask {
    int32_t room, chan, blk;
};

struct RoomDesc {
    double fs_over_c;          // fs / c0
    double r;                  // reflection coefficient of the draws (Eq. 2 or override)
    double centre[3];          // mean microphone (sphere centre of Sec. III-B)
    int64_t out_off;           // first float of the room in the packed output
    int32_t T, n_src, n_mic;
    int32_t src0, mic0;        // first global source / microphone row
    int32_t item0, n_item;     // range in room_items
    int32_t chan0;             // first (source, mic) channel of the room
    double fs, c;              // sample rate and speed of sound (early window index)
    int64_t early_off;         // first float of the room's early windows
    int32_t early_pre, early_post;   // ceil(6 fs / 1000), ceil(50 fs / 1000) (Eq. 9)
    // multi-rate plans only (hr = 0 otherwise).  T, fs_over_c and out_off
    // above then describe the intermediate signal at r_l fs.
    double hr;                 // r_h fs (exact)
    double lm1;                // L - 1, L = ceil(T60 r_h fs)
    double rl, rh;             // r_l, r_h
    double hp_b0, hp_a1, hp_a2;   // 80 Hz Butterworth high-pass: b = b0 (1, -2, 1), a = (1, a1, a2)
    double phi[4];             // state transition of the high-pass over one chunk (row-major)
    double phi_sub[8][4];      // the same over j sub-chunks of kHpSub samples, j = 0 .. 7
    int64_t out2_off;          // first float of the room in the output at fs
    int64_t chunk0;            // first high-pass chunk of the room
    int32_t T_out;             // ceil(T60 fs)
    int32_t n_chunks;          // high-pass chunks per channel
};

constexpr int kHpChunk = 256;         // intermediate samples per high-pass chunk
constexpr int kHpEndChunks = 32;      // chunks per block of the high-pass state pass
constexpr int kHpSub = 32;            // samples per sub-chunk (one thread's run of the recursion)
constexpr int kMaxRl = 12;            // largest r_l a multi-rate plan accepts
// Decimation on the matrix cores: a workgroup of kDmThreads takes kDmBlocks
// blocks of 256 outputs (one per wave).  The filter matrix of an r_l, W[i][q]
// = k[i r_l + half + pad - q] (16 x K, K <= 32 kDmMaxSteps), is kept per r_l
// (1 .. kMaxRl) as fp16 hi / lo fragments: kDmFragWords 32-bit words each.
constexpr int kDmBlocks = 4;
constexpr int kDmThreads = 64 * kDmBlocks;
constexpr int kDmOut = 256 * kDmBlocks;          // outputs per workgroup tile
constexpr int kDmMaxSteps = 37;                  // ceil((7 + 15 r_l + 2 half + 1) / 32) at r_l = 12
constexpr int kDmFragWords = kDmMaxSteps * 2 * 64 * 4;

struct SrcDesc {
    double d0, q, ct, rrmax;   // |src - centre|, c0T60 / d0, c0T60, RR_max (Eq. 5)
    double pos[3];             // source position used by the draws
    uint32_t key0, key1;       // Philox key from the room seed
    int32_t room, s_local;
    int32_t n_img;             // I + 1 rows (row 0 = direct path)
    int32_t pad0;
    int64_t img_off;           // first row in the image table
};

struct WorkItem {
    int32_t src;               // global source index
    int32_t mic0;              // first microphone of the group (room-local)
    int32_t n_mic;             // microphones in the group
    int32_t t0;                // first output sample of the tile
    int32_t len;               // samples of the tile (the last tile may reach past T)
    int32_t full;              // 1 if the tile covers [0, T): every image is in range
    int32_t pad0, pad1;
};

FR_HD const DescHeader* hdr(const void* blob) { return reinterpret_cast<const DescHeader*>(blob); }
FR_HD const RoomDesc* rooms(const void* blob) {
    return reinterpret_cast<const RoomDesc*>(reinterpret_cast<const char*>(blob) + hdr(blob)->room_bytes);
}
FR_HD const SrcDesc* srcs(const void* blob) {
    return reinterpret_cast<const SrcDesc*>(reinterpret_cast<const char*>(blob) + hdr(blob)->src_bytes);
}
FR_HD const WorkItem* items(const void* blob) {
    return reinterpret_cast<const WorkItem*>(reinterpret_cast<const char*>(blob) + hdr(blob)->item_bytes);
}
FR_HD const int32_t* room_items(const void* blob) {
    return reinterpret_cast<const int32_t*>(reinterpret_cast<const char*>(blob) + hdr(blob)->room_items_bytes);
}
FR_HD const int32_t* src_order(const void* blob) {
    return reinterpret_cast<const int32_t*>(reinterpret_cast<const char*>(blob) + hdr(blob)->src_order_bytes);
}
FR_HD const HpTask* hp_tasks(const void* blob) {
    return reinterpret_cast<const HpTask*>(reinterpret_cast<const char*>(blob) + hdr(blob)->hp_task_bytes);
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Round: multiply words 0
// and 2 by M0, M1 into 64-bit products; new state (hi(M1 x2) ^ x1 ^ k0,
// lo(M1 x2), hi(M0 x0) ^ x3 ^ k1, lo(M0 x0)); the key advances by the Weyl
// increments between rounds.
// ---------------------------------------------------------------------------
constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

FR_HD void philox4x32_10(uint32_t x[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += kPhiloxW0;
            k1 += kPhiloxW1;
        }
        const uint64_t p0 = static_cast<uint64_t>(kPhiloxM0) * x[0];
        const uint64_t p1 = static_cast<uint64_t>(kPhiloxM1) * x[2];
        const uint32_t y0 = static_cast<uint32_t>(p1 >> 32) ^ x[1] ^ k0;
        const uint32_t y1 = static_cast<uint32_t>(p1);
        const uint32_t y2 = static_cast<uint32_t>(p0 >> 32) ^ x[3] ^ k1;
        const uint32_t y3 = static_cast<uint32_t>(p0);
        x[0] = y0;
        x[1] = y1;
        x[2] = y2;
        x[3] = y3;
    }
}

// ---------------------------------------------------------------------------
// Bit-level FP64 helpers.
// ---------------------------------------------------------------------------
FR_HD uint64_t dbits(double x) {
    union { double d; uint64_t u; } v;
    v.d = x;
    return v.u;
}
FR_HD double bitsd(uint64_t u) {
    union { double d; uint64_t u; } v;
    v.u = u;
    return v.d;
}
FR_HD double next_up(double x) { return bitsd(dbits(x) + 1); }      // x > 0 finite
FR_HD double next_down(double x) { return bitsd(dbits(x) - 1); }    // x > 0, not the smallest

FR_HD uint64_t mul64hi(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __umul64hi(a, b);
#else
    return static_cast<uint64_t>((static_cast<unsigned __int128>(a) * b) >> 64);
#endif
}

FR_HD double fma_d(double a, double b, double c) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_fma(a, b, c);
#else
    return __builtin_fma(a, b, c);
#endif
}

// Correctly rounded square root of a positive normal double.  The hardware
// sequence gives a value within one ulp; the Tuckerman test then moves it to
// the nearest double: y is RN(sqrt(x)) iff y (y - ulp-) < x <= y (y + ulp+),
// each product compared with x exactly through the sign of one FMA.
FR_HD double sqrt_rn(double x) {
    double y = __builtin_sqrt(x);
#pragma unroll 1
    for (int it = 0; it < 4; ++it) {
        const double up = next_up(y);
        if (fma_d(y, up, -x) < 0.0) {          // x > y * next_up(y): y too small
            y = up;
            continue;
        }
        const double dn = next_down(y);
        if (fma_d(y, dn, -x) >= 0.0) {         // x <= y * next_down(y): y too large
            y = dn;
            continue;
        }
        break;
    }
    return y;
}

// Sign of a - ((2Y + 1) 2^(e - 1))^3 for a = A 2^ea, the cube of the midpoint
// between y = Y 2^e (Y a 53-bit integer) and its successor, compared exactly
// in 256-bit integer arithmetic.  Returns +1, 0 or -1.
FR_HD int cmp_cube_midpoint(uint64_t A, int ea, uint64_t Y, int e) {
    const uint64_t N = 2 * Y + 1;                      // < 2^54
    // N^3 as limbs c0..c2 (little endian)
    const uint64_t sq_lo = N * N, sq_hi = mul64hi(N, N);   // N^2 < 2^108
    const uint64_t t0 = sq_lo * N, t1 = mul64hi(sq_lo, N); // sq_lo * N
    const uint64_t u0 = sq_hi * N, u1 = mul64hi(sq_hi, N); // sq_hi * N (<< 64)
    uint64_t c[4];
    c[0] = t0;
    c[1] = t1 + u0;
    c[2] = u1 + (c[1] < t1 ? 1u : 0u);
    c[3] = 0;
    // A * 2^(ea - 3(e - 1)) against N^3 * 2^0, or N^3 shifted when negative
    const int s = ea - 3 * (e - 1);
    uint64_t l[4] = {0, 0, 0, 0};
    uint64_t r[4] = {c[0], c[1], c[2], c[3]};
    if (s >= 0) {
        if (s >= 256) return 1;
        const int w = s >> 6, b = s & 63;
        l[w] = A << b;
        if (b != 0 && w + 1 < 4) l[w + 1] = A >> (64 - b);
        if (w + 1 < 4 && b == 0) l[w + 1] = 0;
    } else {
        const int t = -s;
        if (t >= 96) return -1;                        // N^3 << t exceeds 2^256 > A
        const int w = t >> 6, b = t & 63;
        uint64_t sh[4] = {0, 0, 0, 0};
        for (int k = 3; k >= 0; --k) {
            const int src = k - w;
            uint64_t v = 0;
            if (src >= 0) {
                v = c[src] << b;
                if (b != 0 && src - 1 >= 0) v |= c[src - 1] >> (64 - b);
            }
            sh[k] = v;
        }
        for (int k = 0; k < 4; ++k) r[k] = sh[k];
        l[0] = A;
    }
    for (int k = 3; k >= 0; --k) {
        if (l[k] > r[k]) return 1;
        if (l[k] < r[k]) return -1;
    }
    return 0;
}

// 53-bit integer mantissa and exponent of a positive normal double:
// x = M 2^e with 2^52 <= M < 2^53.
FR_HD void decompose(double x, uint64_t* M, int* e) {
    const uint64_t u = dbits(x);
    *M = (u & ((uint64_t(1) << 52) - 1)) | (uint64_t(1) << 52);
    *e = static_cast<int>((u >> 52) & 0x7FF) - 1075;
}

// Reciprocal accurate to about one ulp (device: hardware estimate plus one
// Newton step; host: division).  Only used where the exact checks below
// absorb its error.
FR_HD double approx_rcp(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(x);
    r = fma_d(fma_d(-x, r, 1.0), r, r);
    return r;
#else
    return 1.0 / x;
#endif
}

// Exact-ish residual m - y^3 from error-free products: y^2 = p_hi + p_lo and
// p_hi y = c_hi + c_lo exactly; m - c_hi is exact (Sterbenz), so only the
// tiny term p_lo y is rounded.
FR_HD double cube_residual(double m, double y) {
    const double p_hi = y * y;
    const double p_lo = fma_d(y, y, -p_hi);
    const double c_hi = p_hi * y;
    const double c_lo = fma_d(p_hi, y, -c_hi);
    return ((m - c_hi) - c_lo) - p_lo * y;
}

// Correctly rounded cube root of a positive normal double (the inverse CDF of
// Eq. 3).  The argument is scaled into m in [1, 8) by a multiple of 3 in the
// exponent; a float seed, one Newton step and one step from the exact
// residual give y within about half an ulp of cbrt(m).  The residual then
// proves y is the nearest double unless cbrt(m) lies within 1e-6 ulp of a
// rounding midpoint; those rare cases are settled by exact 256-bit integer
// comparisons against the cubes of the midpoints.
FR_HD double cbrt_rn(double a) {
    uint64_t A;
    int ea;
    decompose(a, &A, &ea);
    const int eb = ea + 52;                            // a = (A / 2^52) 2^eb, A/2^52 in [1, 2)
    int q3 = eb >= 0 ? eb / 3 : -((-eb + 2) / 3);      // floor(eb / 3)
    const double m = bitsd((dbits(a) & ~(uint64_t(0x7FF) << 52)) |
                           (uint64_t(1023 + (eb - 3 * q3)) << 52));   // in [1, 8)
    double y = static_cast<double>(cbrtf(static_cast<float>(m)));
    y = y - (y * y * y - m) * approx_rcp(3.0 * y * y);                 // ~1e-14
    const double inv3y2 = approx_rcp(3.0 * y * y);
    y = y + cube_residual(m, y) * inv3y2;                              // ~0.5 ulp
    // offset of cbrt(m) from y in ulps of y (y in [1, 2): ulp = 2^-52)
    const double t = cube_residual(m, y) * approx_rcp(3.0 * y * y) * 4503599627370496.0;
    const double pow2 = bitsd(uint64_t(1023 + q3) << 52);               // exact scaling
    if (t > -0.499999 && t < 0.499999 && y >= 1.0 && y < 2.0) return y * pow2;
    y = y * pow2;
#pragma unroll 1
    for (int it = 0; it < 6; ++it) {
        uint64_t Y;
        int ey;
        decompose(y, &Y, &ey);
        if (cmp_cube_midpoint(A, ea, Y, ey) > 0) {     // a above the upper midpoint
            y = next_up(y);
            continue;
        }
        const double yd = next_down(y);
        decompose(yd, &Y, &ey);
        if (cmp_cube_midpoint(A, ea, Y, ey) < 0) {     // a below the lower midpoint
            y = yd;
            continue;
        }
        break;
    }
    return y;
}

// sin(pi x) and cos(pi x) for |x| <= 2 where x is exact: x = n/2 + r with
// |r| <= 1/4 exactly, then Taylor series of sin and cos at pi r (|pi r| <=
// pi/4; terms to degree 17/18, remainder below 1e-19) and a quarter-turn
// rotation by n.
FR_HD void sincospi_d(double x, double* s_out, double* c_out) {
    const double n = __builtin_rint(2.0 * x);
    const double r = x - 0.5 * n;                      // exact
    const double z = r * 3.141592653589793238;
    const double z2 = z * z;
    double ps = 2.8114572543455206e-15;                // 1/17!
    ps = fma_d(ps, -z2, 7.647163731819816e-13);        // 1/15!
    ps = fma_d(ps, -z2, 1.6059043836821613e-10);       // 1/13!
    ps = fma_d(ps, -z2, 2.505210838544172e-08);        // 1/11!
    ps = fma_d(ps, -z2, 2.7557319223985893e-06);       // 1/9!
    ps = fma_d(ps, -z2, 1.984126984126984e-04);        // 1/7!
    ps = fma_d(ps, -z2, 8.333333333333333e-03);        // 1/5!
    ps = fma_d(ps, -z2, 1.6666666666666666e-01);       // 1/3!
    ps = fma_d(ps, -z2, 1.0);
    const double sr = z * ps;
    double pc = 1.5619206968586225e-16;                // 1/18!
    pc = fma_d(pc, -z2, 4.779477332387385e-14);        // 1/16!
    pc = fma_d(pc, -z2, 1.1470745597729725e-11);       // 1/14!
    pc = fma_d(pc, -z2, 2.08767569878681e-09);         // 1/12!
    pc = fma_d(pc, -z2, 2.755731922398589e-07);        // 1/10!
    pc = fma_d(pc, -z2, 2.48015873015873e-05);         // 1/8!
    pc = fma_d(pc, -z2, 1.388888888888889e-03);        // 1/6!
    pc = fma_d(pc, -z2, 4.1666666666666664e-02);       // 1/4!
    pc = fma_d(pc, -z2, 0.5);                          // 1/2!
    const double cr = fma_d(pc, -z2, 1.0);
    const int q = static_cast<int>(n) & 3;
    // sin(pi r + q pi/2), cos(pi r + q pi/2)
    const double s = (q == 0) ? sr : (q == 1) ? cr : (q == 2) ? -sr : -cr;
    const double c = (q == 0) ? cr : (q == 1) ? -sr : (q == 2) ? -cr : sr;
    *s_out = s;
    *c_out = c;
}

}  // namespace framrir
