// Host planner of the FRAM-RIR library: validation, per-room and per-source
// scalars (Sec. II, III-A, III-C; Eq. 2, Eq. 5), image counts, the device
// descriptor blob and the render work items.  No device calls here.
//
// Build with -ffp-contract=off: every FP64 expression below is rounded one
// operation at a time in the order written, so the scalars that feed the
// bit-exact draws are a function of the inputs and the C library alone.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/framrir.h"
#include "framrir_internal.h"
#include "plan_internal.h"

using namespace framrir;

// ---------------------------------------------------------------------------
// Error reporting
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

int fr_fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = std::string(framrir_strerror(code)) + ": " + buf;
    return code;
}

extern "C" int framrir_last_error_detail(char* buf, size_t n) {
    if (buf && n > 0) {
        const size_t k = std::min(n - 1, g_last_error.size());
        std::memcpy(buf, g_last_error.data(), k);
        buf[k] = '\0';
    }
    return static_cast<int>(g_last_error.size());
}

extern "C" const char* framrir_strerror(int code) {
    switch (code) {
        case FRAMRIR_OK: return "ok";
        case FRAMRIR_E_INVALID_ARG: return "invalid argument";
        case FRAMRIR_E_GEOMETRY: return "invalid geometry";
        case FRAMRIR_E_RANGE: return "value out of range";
        case FRAMRIR_E_WORKSPACE: return "workspace too small";
        case FRAMRIR_E_DEVICE: return "device error";
        case FRAMRIR_E_UNSUPPORTED: return "unsupported";
        default: return "unknown error";
    }
}

extern "C" int framrir_version(void) { return (1 << 16) | 0; }

// ---------------------------------------------------------------------------
// Scalars
// ---------------------------------------------------------------------------
namespace {

bool finite3(const double* p) { return std::isfinite(p[0]) && std::isfinite(p[1]) && std::isfinite(p[2]); }

bool strictly_inside(const double* p, const double* size) {
    for (int k = 0; k < 3; ++k)
        if (!(p[k] > 0.0 && p[k] < size[k])) return false;
    return true;
}

// R = V / S of the empty shoebox (Sec. III-A); r from Eq. 2 as printed.
double eyring_r(const double* size, double rt60) {
    const double lx = size[0], ly = size[1], lz = size[2];
    const double volume = (lx * ly) * lz;
    const double area = 2.0 * ((lx * ly + lx * lz) + ly * lz);
    const double big_r = volume / area;
    const double x = (0.16 * big_r) / rt60;
    const double eps = 1.0 - std::exp(-x);
    return std::sqrt(1.0 - eps * eps);
}

}  // namespace

// ---------------------------------------------------------------------------
// Plan
// ---------------------------------------------------------------------------
extern "C" int framrir_plan_create(const framrir_room* rooms_in, int32_t n_rooms, const framrir_params* prm_in,
                                   const framrir_launch* launch_in, const double* src, const double* mic,
                                   framrir_plan** out) {
    if (!out) return fr_fail(FRAMRIR_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!rooms_in || !src || !mic) return fr_fail(FRAMRIR_E_INVALID_ARG, "rooms, src and mic must be non-NULL");
    if (n_rooms <= 0) return fr_fail(FRAMRIR_E_INVALID_ARG, "n_rooms = %d must be >= 1", n_rooms);

    framrir_params prm;
    if (prm_in) {
        prm = *prm_in;
    } else {
        prm = framrir_params{0.25, 1.0, -2.0, 2.0, 0.25, 1024, 4096, FRAMRIR_TAPS, 0u};
    }
    framrir_launch launch = launch_in ? *launch_in : framrir_launch{131072, 1024, 0, 8, 4, 0, 0, 0};
    if (launch.max_mic_group == 0) launch.max_mic_group = 8;
    if (launch.waves_per_simd == 0) launch.waves_per_simd = 4;
    if (launch.bwd_wg_threads == 0) launch.bwd_wg_threads = launch.wg_threads;

    // ---- method parameters
    if (!(std::isfinite(prm.alpha) && std::isfinite(prm.beta) && std::isfinite(prm.a) && std::isfinite(prm.b) &&
          std::isfinite(prm.tau)))
        return fr_fail(FRAMRIR_E_INVALID_ARG, "non-finite method parameter");
    if (!(prm.alpha >= 0.0 && prm.alpha < prm.beta && prm.beta <= 1.0))
        return fr_fail(FRAMRIR_E_RANGE, "need 0 <= alpha < beta <= 1 (alpha=%g beta=%g)", prm.alpha, prm.beta);
    if (!(prm.a <= prm.b)) return fr_fail(FRAMRIR_E_RANGE, "need a <= b (a=%g b=%g)", prm.a, prm.b);
    int32_t tau_code;
    if (prm.tau == 0.25) tau_code = kTauQuarter;
    else if (prm.tau == 0.5) tau_code = kTauHalf;
    else if (prm.tau == 1.0) tau_code = kTauOne;
    else return fr_fail(FRAMRIR_E_RANGE, "tau must be 0.25, 0.5 or 1 (got %g)", prm.tau);
    if (!(prm.img_lo >= 0 && prm.img_lo <= prm.img_hi && prm.img_hi <= 65535))
        return fr_fail(FRAMRIR_E_RANGE, "need 0 <= img_lo <= img_hi <= 65535 (%d, %d)", prm.img_lo, prm.img_hi);
    if (prm.taps != FRAMRIR_TAPS) return fr_fail(FRAMRIR_E_UNSUPPORTED, "taps must be 81 (got %d)", prm.taps);
    if ((prm.flags & ~FRAMRIR_FLAG_MULTIRATE) != 0u)
        return fr_fail(FRAMRIR_E_UNSUPPORTED, "unknown flags 0x%x", prm.flags);
    const bool multirate = (prm.flags & FRAMRIR_FLAG_MULTIRATE) != 0u;

    // ---- launch shape
    if (launch.wg_threads < 64 || launch.wg_threads > 1024 || launch.wg_threads % 64 != 0)
        return fr_fail(FRAMRIR_E_RANGE, "wg_threads must be a multiple of 64 in [64, 1024] (got %d)",
                       launch.wg_threads);
    if (launch.lds_bytes < 4096 || launch.lds_bytes > kMaxDynLdsBytes || launch.lds_bytes % 16 != 0)
        return fr_fail(FRAMRIR_E_RANGE, "lds_bytes must be a multiple of 16 in [4096, %d] (got %d)",
                       kMaxDynLdsBytes, launch.lds_bytes);
    if (launch.waves_per_simd != 4 && launch.waves_per_simd != 8)
        return fr_fail(FRAMRIR_E_UNSUPPORTED, "waves_per_simd must be 4 or 8 (got %d)", launch.waves_per_simd);
    if (launch.wg_threads != 256 && launch.wg_threads != 512 && launch.wg_threads != 1024)
        return fr_fail(FRAMRIR_E_UNSUPPORTED, "wg_threads must be 256, 512 or 1024 (got %d)", launch.wg_threads);
    const int render_static = launch.render_path == 1 ? kMomStaticLds : render_static_lds(launch.wg_threads);
    if (launch.lds_bytes + render_static > kLdsPerCu)
        return fr_fail(FRAMRIR_E_RANGE, "lds_bytes + the render's static LDS (%d) must not exceed %d (got %d)",
                       render_static, kLdsPerCu, launch.lds_bytes);
    if (launch.bwd_wg_threads != 256 && launch.bwd_wg_threads != 512 && launch.bwd_wg_threads != 1024)
        return fr_fail(FRAMRIR_E_UNSUPPORTED, "bwd_wg_threads must be 0, 256, 512 or 1024 (got %d)",
                       launch.bwd_wg_threads);
    if (launch.lds_bytes < 28 * std::max(launch.wg_threads, launch.bwd_wg_threads))
        return fr_fail(FRAMRIR_E_RANGE, "lds_bytes must be >= 28 * the workgroup size (backward reduction)");
    if (launch.max_mic_group < 1 || launch.max_mic_group > kMaxMicGroup)
        return fr_fail(FRAMRIR_E_RANGE, "max_mic_group must be in [1, %d]", kMaxMicGroup);
    if (launch.grid_wgs < 0 || launch.bwd_grid_wgs < 0)
        return fr_fail(FRAMRIR_E_RANGE, "grid_wgs and bwd_grid_wgs must be >= 0");
    if (launch.render_path != 0 && launch.render_path != 1)
        return fr_fail(FRAMRIR_E_UNSUPPORTED, "render_path must be 0 (scatter) or 1 (bin moments) (got %d)",
                       launch.render_path);
    if (launch.render_path == 1 && launch.waves_per_simd != 4)
        return fr_fail(FRAMRIR_E_UNSUPPORTED, "the bin-moment render runs at 4 waves per SIMD (its matrix-core "
                                              "FIR needs more than 64 registers)");

    framrir_plan* plan = new (std::nothrow) framrir_plan();
    if (!plan) return fr_fail(FRAMRIR_E_INVALID_ARG, "out of host memory");
    plan->launch = launch;
    plan->prm = prm;

    std::vector<RoomDesc>& rd = plan->rooms;
    std::vector<SrcDesc>& sd = plan->srcs;
    rd.resize(n_rooms);
    int64_t out_off = 0, img_off = 0, early_off = 0, out2_off = 0, chunk_row = 0;
    int32_t chan_row = 0, max_early = 0, max_room_chan = 0, max_chunks = 0, max_out_tiles = 0, max_rl = 0;
    int32_t src_row = 0, mic_row = 0, max_img = 0, max_T = 0;

    for (int32_t b = 0; b < n_rooms; ++b) {
        const framrir_room& rm = rooms_in[b];
        if (!finite3(rm.size) || !std::isfinite(rm.rt60) || !std::isfinite(rm.fs) || !std::isfinite(rm.c)) {
            delete plan;
            return fr_fail(FRAMRIR_E_INVALID_ARG, "room %d: non-finite size, T60, fs or c", b);
        }
        if (!(rm.size[0] > 0.0 && rm.size[1] > 0.0 && rm.size[2] > 0.0)) {
            delete plan;
            return fr_fail(FRAMRIR_E_GEOMETRY, "room %d: dimensions must be > 0", b);
        }
        if (!(rm.rt60 > 0.0 && rm.fs > 0.0 && rm.c > 0.0)) {
            delete plan;
            return fr_fail(FRAMRIR_E_RANGE, "room %d: T60, fs and c must be > 0", b);
        }
        if (rm.n_src < 1 || rm.n_mic < 1 || rm.n_mic > FRAMRIR_MAX_MICS) {
            delete plan;
            return fr_fail(FRAMRIR_E_INVALID_ARG, "room %d: need n_src >= 1 and 1 <= n_mic <= %d", b,
                           FRAMRIR_MAX_MICS);
        }
        const double t_samples = std::ceil(rm.rt60 * rm.fs);   // T = ceil(T60 fs)
        if (!(t_samples >= 1.0 && t_samples <= 2147483647.0 - 256.0)) {
            delete plan;
            return fr_fail(FRAMRIR_E_RANGE, "room %d: T = ceil(T60 fs) out of range", b);
        }
        const int32_t T = static_cast<int32_t>(t_samples);
        // the render's rate and length: fs and T, or r_l fs and T_l for the
        // paper-literal multi-rate rendering (Sec. II, Sec. III-D)
        double fs_r = rm.fs, hr = 0.0, lm1 = 0.0;
        int32_t T_r = T, rh = 0, rl = 0;
        if (multirate) {
            const double rhd = std::floor(1.0e6 / rm.fs);
            rh = rhd >= 1.0 && rhd < 2147483647.0 ? static_cast<int32_t>(rhd) : 0;
            rl = 0;
            while (static_cast<int64_t>(rl + 1) * (rl + 1) <= rh) ++rl;   // floor(sqrt(r_h)) in integers
            if (!(rl > 1 && rl <= kMaxRl)) {
                delete plan;
                return fr_fail(FRAMRIR_E_RANGE, "room %d: multi-rate needs 1 < r_l <= %d (fs = %g gives r_h = %d)", b,
                               kMaxRl, rm.fs, rh);
            }
            hr = rh * rm.fs;
            const double big_l = std::ceil(rm.rt60 * hr);
            fs_r = rl * rm.fs;
            const double tl = std::ceil(rm.rt60 * fs_r);
            if (!(big_l >= 1.0 && big_l <= 9007199254740992.0 && tl >= 1.0 && tl <= 2147483647.0 - 256.0)) {
                delete plan;
                return fr_fail(FRAMRIR_E_RANGE, "room %d: multi-rate lengths out of range", b);
            }
            lm1 = big_l - 1.0;
            T_r = static_cast<int32_t>(tl);
        }
        double r;
        if (std::isnan(rm.r_override)) {
            r = eyring_r(rm.size, rm.rt60);
        } else {
            r = rm.r_override;
        }
        if (!(r > 0.0 && r < 1.0)) {
            delete plan;
            return fr_fail(FRAMRIR_E_RANGE, "room %d: reflection coefficient r = %.17g not in (0, 1)", b, r);
        }
        // microphones: inside, and the centre in microphone order (Sec. III-B)
        const double* mics = mic + 3 * static_cast<int64_t>(mic_row);
        double cx = 0.0, cy = 0.0, cz = 0.0;
        for (int32_t m = 0; m < rm.n_mic; ++m) {
            const double* p = mics + 3 * m;
            if (!finite3(p)) {
                delete plan;
                return fr_fail(FRAMRIR_E_INVALID_ARG, "room %d mic %d: non-finite position", b, m);
            }
            if (!strictly_inside(p, rm.size)) {
                delete plan;
                return fr_fail(FRAMRIR_E_GEOMETRY, "room %d mic %d: not strictly inside the room", b, m);
            }
            cx += p[0];
            cy += p[1];
            cz += p[2];
        }
        const double nm = static_cast<double>(rm.n_mic);
        RoomDesc& R = rd[b];
        std::memset(&R, 0, sizeof(R));
        R.fs_over_c = fs_r / rm.c;
        R.r = r;
        R.centre[0] = cx / nm;
        R.centre[1] = cy / nm;
        R.centre[2] = cz / nm;
        R.out_off = out_off;
        R.T = T_r;
        R.T_out = T;
        R.out2_off = multirate ? out2_off : out_off;
        R.n_src = rm.n_src;
        R.n_mic = rm.n_mic;
        R.src0 = src_row;
        R.mic0 = mic_row;
        R.chan0 = chan_row;
        R.fs = rm.fs;
        R.c = rm.c;
        R.early_off = early_off;
        R.early_pre = static_cast<int32_t>(std::ceil(6.0 * rm.fs / 1000.0));
        R.early_post = static_cast<int32_t>(std::ceil(50.0 * rm.fs / 1000.0));
        if (multirate) {
            R.hr = hr;
            R.lm1 = lm1;
            R.rl = rl;
            R.rh = rh;
            // second-order Butterworth high-pass, bilinear with the cut-off
            // prewarped to 80 Hz at r_l fs: b = b0 (1, -2, 1), a = (1, a1, a2)
            const double k = std::tan(M_PI * 80.0 / fs_r);
            const double norm = 1.0 + std::sqrt(2.0) * k + k * k;
            R.hp_b0 = 1.0 / norm;
            R.hp_a1 = 2.0 * (k * k - 1.0) / norm;
            R.hp_a2 = (1.0 - std::sqrt(2.0) * k + k * k) / norm;
            // phi = M^kHpChunk and phi_sub[j] = M^(j kHpSub), M = [[-a1, -a2], [1, 0]]
            // mapping (y[n-1], y[n-2]) of the unforced recurrence to (y[n], y[n-1])
            const auto mat_pow = [&](int n, double* out) {
                double m[4] = {-R.hp_a1, -R.hp_a2, 1.0, 0.0}, acc[4] = {1.0, 0.0, 0.0, 1.0};
                for (int e = n; e > 0; e >>= 1) {
                    double t[4];
                    if (e & 1) {
                        t[0] = acc[0] * m[0] + acc[1] * m[2];
                        t[1] = acc[0] * m[1] + acc[1] * m[3];
                        t[2] = acc[2] * m[0] + acc[3] * m[2];
                        t[3] = acc[2] * m[1] + acc[3] * m[3];
                        std::memcpy(acc, t, sizeof(t));
                    }
                    t[0] = m[0] * m[0] + m[1] * m[2];
                    t[1] = m[0] * m[1] + m[1] * m[3];
                    t[2] = m[2] * m[0] + m[3] * m[2];
                    t[3] = m[2] * m[1] + m[3] * m[3];
                    std::memcpy(m, t, sizeof(t));
                }
                std::memcpy(out, acc, sizeof(acc));
            };
            mat_pow(kHpChunk, R.phi);
            static_assert(kHpChunk == 8 * kHpSub, "eight sub-chunks per chunk");
            for (int j = 0; j < 8; ++j) mat_pow(j * kHpSub, R.phi_sub[j]);
            R.n_chunks = (T_r + kHpChunk - 1) / kHpChunk;
            R.chunk0 = chunk_row;
        }
        const double ct = rm.c * rm.rt60;
        const double log10_r = std::log10(r);
        const double log10_ct = std::log10(ct);
        for (int32_t s = 0; s < rm.n_src; ++s) {
            const double* p = src + 3 * static_cast<int64_t>(src_row + s);
            if (!finite3(p)) {
                delete plan;
                return fr_fail(FRAMRIR_E_INVALID_ARG, "room %d source %d: non-finite position", b, s);
            }
            if (!strictly_inside(p, rm.size)) {
                delete plan;
                return fr_fail(FRAMRIR_E_GEOMETRY, "room %d source %d: not strictly inside the room", b, s);
            }
            for (int32_t m = 0; m < rm.n_mic; ++m) {
                const double* q = mics + 3 * m;
                const double ex = p[0] - q[0], ey = p[1] - q[1], ez = p[2] - q[2];
                if (!((ex * ex + ey * ey) + ez * ez > 1e-18)) {
                    delete plan;
                    return fr_fail(FRAMRIR_E_GEOMETRY, "room %d source %d coincides with mic %d", b, s, m);
                }
            }
            const double dx = p[0] - R.centre[0];
            const double dy = p[1] - R.centre[1];
            const double dz = p[2] - R.centre[2];
            const double d0 = std::sqrt((dx * dx + dy * dy) + dz * dz);
            if (!(d0 > 0.0)) {
                delete plan;
                return fr_fail(FRAMRIR_E_GEOMETRY, "room %d source %d: at the array centre (d0 = 0)", b, s);
            }
            if (!(d0 < ct)) {
                delete plan;
                return fr_fail(FRAMRIR_E_GEOMETRY, "room %d source %d: d0 = %g >= c0 T60 = %g", b, s, d0, ct);
            }
            SrcDesc S;
            std::memset(&S, 0, sizeof(S));
            S.d0 = d0;
            S.ct = ct;
            S.q = ct / d0;
            // Eq. 5, clamped below at 1 (spreading alone may already reach -60 dB)
            double rr = ((log10_ct - std::log10(d0)) - 3.0) / log10_r;
            S.rrmax = rr > 1.0 ? rr : 1.0;
            S.pos[0] = p[0];
            S.pos[1] = p[1];
            S.pos[2] = p[2];
            S.key0 = static_cast<uint32_t>(rm.seed & 0xFFFFFFFFu);
            S.key1 = static_cast<uint32_t>(rm.seed >> 32);
            S.room = b;
            S.s_local = s;
            // image count from the header counter (0, s, 1, 0)
            uint32_t x[4] = {0u, static_cast<uint32_t>(s), 1u, 0u};
            philox4x32_10(x, S.key0, S.key1);
            const uint64_t span = static_cast<uint64_t>(prm.img_hi - prm.img_lo + 1);
            const int32_t I = prm.img_lo + static_cast<int32_t>((static_cast<uint64_t>(x[0]) * span) >> 32);
            S.n_img = I + 1;
            S.img_off = img_off;
            img_off += S.n_img;
            max_img = std::max(max_img, S.n_img);
            sd.push_back(S);
        }
        out_off += static_cast<int64_t>(rm.n_src) * rm.n_mic * T_r;
        const int32_t n_chan_room = rm.n_src * rm.n_mic;
        if (multirate) {
            out2_off += static_cast<int64_t>(n_chan_room) * T;
            chunk_row += static_cast<int64_t>(n_chan_room) * R.n_chunks;
            max_chunks = std::max(max_chunks, R.n_chunks);
            max_out_tiles = std::max(max_out_tiles, (T + kDmOut - 1) / kDmOut);
            max_rl = std::max(max_rl, rl);
        }
        early_off += static_cast<int64_t>(n_chan_room) * (R.early_pre + R.early_post + 1);
        chan_row += n_chan_room;
        max_early = std::max(max_early, R.early_pre + R.early_post + 1);
        max_room_chan = std::max(max_room_chan, n_chan_room);
        src_row += rm.n_src;
        mic_row += rm.n_mic;
        max_T = std::max(max_T, T_r);
    }

    // ---- work items: per source, microphone groups x time tiles
    std::vector<WorkItem>& it = plan->items;
    std::vector<double> cost;
    for (int32_t b = 0; b < n_rooms; ++b) {
        const RoomDesc& R = rd[b];
        const int n_groups = (R.n_mic + launch.max_mic_group - 1) / launch.max_mic_group;
        for (int g = 0; g < n_groups; ++g) {
            const int m0 = (R.n_mic * g) / n_groups;
            const int m1 = (R.n_mic * (g + 1)) / n_groups;
            const int mg = m1 - m0;
            const int cap = launch.render_path == 1 ? moment_tile_cap(launch.lds_bytes, mg)
                                                    : launch.lds_bytes / 4 / mg - 2 * kHalo;
            if (cap < 64) {
                delete plan;
                return fr_fail(FRAMRIR_E_RANGE, "lds_bytes %d too small for %d microphones", launch.lds_bytes, mg);
            }
            const int n_tiles = (R.T + cap - 1) / cap;
            int len = (R.T + n_tiles - 1) / n_tiles;
            len = (len + 3) & ~3;                       // keep tile starts 16-byte aligned in LDS
            if (len > cap) len = cap & ~3;
            const int n_t = (R.T + len - 1) / len;
            for (int32_t s = 0; s < R.n_src; ++s) {
                const SrcDesc& S = sd[R.src0 + s];
                for (int t = 0; t < n_t; ++t) {
                    WorkItem w;
                    std::memset(&w, 0, sizeof(w));
                    w.src = R.src0 + s;
                    w.mic0 = m0;
                    w.n_mic = mg;
                    w.t0 = t * len;
                    w.len = len;
                    w.full = n_t == 1 ? 1 : 0;
                    it.push_back(w);
                    cost.push_back(static_cast<double>(S.n_img) * mg / n_t + 0.05 * len * mg);
                }
            }
        }
    }
    // longest first (stable), so the dynamic queue of the persistent grid
    // starts the big items early
    std::vector<int32_t> order(it.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = static_cast<int32_t>(k);
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return cost[x] > cost[y]; });
    std::vector<WorkItem> sorted(it.size());
    for (size_t k = 0; k < order.size(); ++k) sorted[k] = it[order[k]];
    it.swap(sorted);
    // per-room item lists in a fixed order (backward reduction)
    std::vector<std::vector<int32_t>> per_room(n_rooms);
    for (size_t k = 0; k < it.size(); ++k) per_room[sd[it[k].src].room].push_back(static_cast<int32_t>(k));
    plan->room_items.clear();
    for (int32_t b = 0; b < n_rooms; ++b) {
        rd[b].item0 = static_cast<int32_t>(plan->room_items.size());
        rd[b].n_item = static_cast<int32_t>(per_room[b].size());
        plan->room_items.insert(plan->room_items.end(), per_room[b].begin(), per_room[b].end());
    }

    // ---- header and blob
    DescHeader H;
    std::memset(&H, 0, sizeof(H));
    H.n_rooms = n_rooms;
    H.n_src = src_row;
    H.n_mic = mic_row;
    H.n_items = static_cast<int32_t>(it.size());
    H.n_img = img_off;
    H.out_floats = out_off;
    H.alpha = prm.alpha;
    H.beta = prm.beta;
    H.a = prm.a;
    H.b = prm.b;
    H.a3 = (prm.alpha * prm.alpha) * prm.alpha;
    H.b3 = (prm.beta * prm.beta) * prm.beta;
    H.beta_minus_alpha = prm.beta - prm.alpha;
    H.b_minus_a = prm.b - prm.a;
    H.tau_code = tau_code;
    H.max_img = max_img;
    H.max_T = max_T;
    H.multirate = multirate ? 1 : 0;
    H.mr_floats = multirate ? out_off : 0;
    if (multirate) H.out_floats = out2_off;
    H.n_chunks = chunk_row;
    H.max_chunks = max_chunks;
    H.max_out_tiles = max_out_tiles;
    H.max_rl = max_rl;
    H.n_chan = chan_row;
    H.early_floats = early_off;
    H.max_early = max_early;
    H.max_room_chan = max_room_chan;
    auto align = [](int64_t v) { return (v + 255) & ~int64_t(255); };
    H.room_bytes = align(sizeof(DescHeader));
    H.src_bytes = align(H.room_bytes + static_cast<int64_t>(sizeof(RoomDesc)) * n_rooms);
    H.item_bytes = align(H.src_bytes + static_cast<int64_t>(sizeof(SrcDesc)) * src_row);
    H.room_items_bytes = align(H.item_bytes + static_cast<int64_t>(sizeof(WorkItem)) * it.size());
    // the preparation takes the sources largest first, so that the workgroups
    // that start last have the least to do
    std::vector<int32_t> src_ord(src_row);
    for (int32_t s = 0; s < src_row; ++s) src_ord[s] = s;
    std::stable_sort(src_ord.begin(), src_ord.end(), [&](int32_t x, int32_t y) { return sd[x].n_img > sd[y].n_img; });
    // When every source's workgroup is resident at once (two per CU), the
    // dispatcher puts workgroups i and i + kCus on one CU, where they share the
    // VALU for the draws: the second half of the order is then reversed, so
    // that the j-th largest source shares its CU with the j-th smallest.
    if (src_row > kCus && src_row <= 2 * kCus) std::reverse(src_ord.begin() + kCus, src_ord.end());
    H.src_order_bytes = align(H.room_items_bytes + static_cast<int64_t>(sizeof(int32_t)) * plan->room_items.size());
    // the high-pass state pass of a multi-rate plan: one task per block of
    // kHpEndChunks chunks of a channel, channel after channel
    std::vector<HpTask> hp;
    if (multirate) {
        for (int32_t b = 0; b < n_rooms; ++b) {
            const int n_blk = (rd[b].n_chunks + kHpEndChunks - 1) / kHpEndChunks;
            for (int ch = 0; ch < rd[b].n_src * rd[b].n_mic; ++ch)
                for (int k = 0; k < n_blk; ++k) hp.push_back(HpTask{b, ch, k});
        }
    }
    H.n_hp_tasks = static_cast<int32_t>(hp.size());
    H.hp_task_bytes = align(H.src_order_bytes + static_cast<int64_t>(sizeof(int32_t)) * src_ord.size());
    const int64_t total = align(H.hp_task_bytes + static_cast<int64_t>(sizeof(HpTask)) * hp.size());
    plan->blob.assign(static_cast<size_t>(total), 0);
    char* base = plan->blob.data();
    std::memcpy(base, &H, sizeof(H));
    std::memcpy(base + H.room_bytes, rd.data(), sizeof(RoomDesc) * rd.size());
    std::memcpy(base + H.src_bytes, sd.data(), sizeof(SrcDesc) * sd.size());
    std::memcpy(base + H.item_bytes, it.data(), sizeof(WorkItem) * it.size());
    std::memcpy(base + H.room_items_bytes, plan->room_items.data(), sizeof(int32_t) * plan->room_items.size());
    std::memcpy(base + H.src_order_bytes, src_ord.data(), sizeof(int32_t) * src_ord.size());
    if (!hp.empty()) std::memcpy(base + H.hp_task_bytes, hp.data(), sizeof(HpTask) * hp.size());
    plan->header = H;

    // ---- workspace
    plan->ws_scale_off = kWsCounterBytes;
    plan->ws_bucket_off = align(plan->ws_scale_off + static_cast<int64_t>(sizeof(float)) * src_row);
    plan->ws_row0_off = align(plan->ws_bucket_off + static_cast<int64_t>(sizeof(int32_t)) * src_row * (kBuckets + 1));
    plan->ws_room_off = align(plan->ws_row0_off + static_cast<int64_t>(sizeof(int32_t)) * src_row);
    plan->ws_rows_off = align(plan->ws_room_off + static_cast<int64_t>(sizeof(int32_t)) * n_rooms);
    plan->ws_bytes = align(plan->ws_rows_off + static_cast<int64_t>(4 * sizeof(double)) * img_off);
    plan->ws_part_off = plan->ws_bytes;
    plan->ws_bwd_bytes = plan->ws_part_off + align(static_cast<int64_t>(sizeof(float)) * kPartialStride * it.size());
    // multi-rate: per high-pass chunk the end deviation y - x of its partial
    // response (2 doubles) and its initial deviation (2 doubles), per
    // sub-chunk the deviation of the chunk's partial response at its start (2
    // doubles), then the decimation fragments
    plan->ws_zend_off = align(plan->ws_bytes);
    plan->ws_init_off = align(plan->ws_zend_off + 16 * chunk_row);
    plan->ws_sub_off = align(plan->ws_init_off + 16 * chunk_row);
    plan->ws_taps_off = align(plan->ws_sub_off + 16 * 8 * chunk_row);
    plan->ws_mr_bytes =
        multirate ? align(plan->ws_taps_off + static_cast<int64_t>(sizeof(uint32_t)) * kDmFragWords * kMaxRl) : 0;
    int32_t grid = launch.grid_wgs;
    if (grid == 0) {
        const int static_lds = launch.render_path == 1 ? kMomStaticLds : render_static_lds(launch.wg_threads);
        const int per_cu_lds = kLdsPerCu / (launch.lds_bytes + static_lds);
        const int per_cu_waves = launch.waves_per_simd * 4 / (launch.wg_threads / 64);
        const int per_cu = std::max(1, std::min(per_cu_lds, per_cu_waves));
        grid = static_cast<int32_t>(std::min<int64_t>(static_cast<int64_t>(it.size()), int64_t(256) * per_cu));
    }
    plan->grid = std::max(1, grid);
    int32_t bwd_grid = launch.bwd_grid_wgs;
    if (bwd_grid == 0 && launch.bwd_wg_threads == launch.wg_threads) bwd_grid = plan->grid;
    if (bwd_grid == 0) {   // the backward's dynamic LDS is max(lds_bytes, 32 x threads); its static LDS is small
        const int lds = std::max(launch.lds_bytes, 32 * launch.bwd_wg_threads) + 2048;
        const int per_cu = std::max(1, std::min(kLdsPerCu / lds, launch.waves_per_simd * 4 / (launch.bwd_wg_threads / 64)));
        bwd_grid = static_cast<int32_t>(std::min<int64_t>(static_cast<int64_t>(it.size()), int64_t(256) * per_cu));
    }
    plan->bwd_grid = std::max(1, bwd_grid);
    *out = plan;
    return FRAMRIR_OK;
}

extern "C" void framrir_plan_destroy(framrir_plan* plan) { delete plan; }

extern "C" int framrir_plan_get_info(const framrir_plan* plan, framrir_plan_info* info) {
    if (!plan || !info) return fr_fail(FRAMRIR_E_INVALID_ARG, "plan and info must be non-NULL");
    const DescHeader& H = plan->header;
    info->n_rooms = H.n_rooms;
    info->n_src = H.n_src;
    info->n_mic = H.n_mic;
    info->n_items = H.n_items;
    info->n_img = H.n_img;
    info->out_floats = H.out_floats;
    info->desc_bytes = static_cast<int64_t>(plan->blob.size());
    info->ws_bytes = plan->ws_bytes;
    info->ws_bwd_bytes = plan->ws_bwd_bytes;
    info->max_T = H.max_T;
    info->max_img = H.max_img;
    info->multirate = H.multirate;
    info->mr_floats = H.mr_floats;
    info->ws_mr_bytes = plan->ws_mr_bytes;
    int64_t blocks = 0;
    if (plan->launch.render_path == 1)
        for (const framrir::WorkItem& w : plan->items)
            blocks += static_cast<int64_t>(w.n_mic) * ((w.len + kMomBlock - 1) / kMomBlock);
    info->fir_blocks = blocks;
    info->n_chan = H.n_chan;
    info->early_floats = H.early_floats;
    return FRAMRIR_OK;
}

extern "C" int framrir_plan_get_early(const framrir_plan* plan, int64_t* early_off, int32_t* width,
                                      int32_t* chan_off) {
    if (!plan) return fr_fail(FRAMRIR_E_INVALID_ARG, "plan is NULL");
    const DescHeader& H = plan->header;
    for (int32_t b = 0; b < H.n_rooms; ++b) {
        const RoomDesc& R = plan->rooms[b];
        if (early_off) early_off[b] = R.early_off;
        if (width) width[b] = R.early_pre + R.early_post + 1;
        if (chan_off) chan_off[b] = R.chan0;
    }
    if (early_off) early_off[H.n_rooms] = H.early_floats;
    if (chan_off) chan_off[H.n_rooms] = H.n_chan;
    return FRAMRIR_OK;
}

extern "C" int framrir_plan_get_arrays(const framrir_plan* plan, int32_t* T, int64_t* out_off, double* r,
                                       int32_t* n_img, int64_t* img_off, double* rrmax, double* d0) {
    if (!plan) return fr_fail(FRAMRIR_E_INVALID_ARG, "plan is NULL");
    const DescHeader& H = plan->header;
    for (int32_t b = 0; b < H.n_rooms; ++b) {
        if (T) T[b] = plan->rooms[b].T_out;
        if (out_off) out_off[b] = plan->rooms[b].out2_off;
        if (r) r[b] = plan->rooms[b].r;
    }
    if (out_off) out_off[H.n_rooms] = H.out_floats;
    for (int32_t s = 0; s < H.n_src; ++s) {
        if (n_img) n_img[s] = plan->srcs[s].n_img;
        if (img_off) img_off[s] = plan->srcs[s].img_off;
        if (rrmax) rrmax[s] = plan->srcs[s].rrmax;
        if (d0) d0[s] = plan->srcs[s].d0;
    }
    if (img_off) img_off[H.n_src] = H.n_img;
    return FRAMRIR_OK;
}

extern "C" const void* framrir_plan_desc(const framrir_plan* plan) {
    return plan ? static_cast<const void*>(plan->blob.data()) : nullptr;
}

// ---------------------------------------------------------------------------
// Host builds of the draw-stage numerics, for checks on machines without a GPU
// ---------------------------------------------------------------------------
extern "C" int framrir_host_cbrt_rn(const double* x, double* y, int64_t n) {
    if (!x || !y || n < 0) return fr_fail(FRAMRIR_E_INVALID_ARG, "bad arguments");
    for (int64_t i = 0; i < n; ++i) {
        const double v = x[i];
        y[i] = (v >= 2.2250738585072014e-308 && std::isfinite(v)) ? cbrt_rn(v) : (v == 0.0 ? 0.0 : NAN);
    }
    return FRAMRIR_OK;
}

extern "C" int framrir_host_sqrt_rn(const double* x, double* y, int64_t n) {
    if (!x || !y || n < 0) return fr_fail(FRAMRIR_E_INVALID_ARG, "bad arguments");
    for (int64_t i = 0; i < n; ++i) {
        const double v = x[i];
        y[i] = (v >= 2.2250738585072014e-308 && std::isfinite(v)) ? sqrt_rn(v) : NAN;
    }
    return FRAMRIR_OK;
}

extern "C" int framrir_host_philox4x32(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t n) {
    if (!ctr || !key || !out || n < 0) return fr_fail(FRAMRIR_E_INVALID_ARG, "bad arguments");
    for (int64_t i = 0; i < n; ++i) {
        uint32_t x[4] = {ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]};
        philox4x32_10(x, key[2 * i], key[2 * i + 1]);
        for (int k = 0; k < 4; ++k) out[4 * i + k] = x[k];
    }
    return FRAMRIR_OK;
}
