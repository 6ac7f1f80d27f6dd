// Library handle and launch-shape tuner (host code).
//
// A handle belongs to one device: on creation it checks that the device is a
// gfx950, looks up the device address of the allocation-free entry point's
// static scratch for that device, and loads the tuning caches.  The tuner
// times framrir_forward (draws, preparation and render) of a caller's batch
// under candidate launch shapes on that device and keeps the fastest per size
// class, in memory and in a JSON file keyed by "architecture|size class".
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/framrir.h"
#include "plan_internal.h"

// defined with the kernels: the per-device scratch address (looked up once)
int framrir_scratch_setup(int device);

namespace {

struct Entry {
    framrir_launch launch;
    double ms;
};

framrir_launch default_launch() { return framrir_launch{131072, 1024, 0, 8, 4, 0, 0, 0}; }

// ---- a small JSON reader for the cache format: an object whose values are
// objects {"launch": {name: integer, ...}, "ms": number}
struct Json {
    const std::string& s;
    size_t i = 0;
    bool ok = true;
    explicit Json(const std::string& text) : s(text) {}
    void ws() {
        while (i < s.size() && std::isspace(static_cast<unsigned char>(s[i]))) ++i;
    }
    bool eat(char c) {
        ws();
        if (i < s.size() && s[i] == c) {
            ++i;
            return true;
        }
        return false;
    }
    std::string str() {
        ws();
        std::string out;
        if (i >= s.size() || s[i] != '"') {
            ok = false;
            return out;
        }
        for (++i; i < s.size() && s[i] != '"'; ++i) {
            if (s[i] == '\\' && i + 1 < s.size()) ++i;
            out.push_back(s[i]);
        }
        if (i >= s.size()) ok = false;
        ++i;
        return out;
    }
    double num() {
        ws();
        const char* b = s.c_str() + i;
        char* e = nullptr;
        const double v = std::strtod(b, &e);
        if (e == b) ok = false;
        i += static_cast<size_t>(e - b);
        return v;
    }
    void skip() {   // any value
        ws();
        if (i >= s.size()) {
            ok = false;
            return;
        }
        if (s[i] == '"') {
            str();
        } else if (s[i] == '{' || s[i] == '[') {
            const char close = s[i] == '{' ? '}' : ']';
            ++i;
            if (eat(close)) return;
            do {
                if (close == '}') {
                    str();
                    if (!eat(':')) ok = false;
                }
                skip();
            } while (ok && eat(','));
            if (!eat(close)) ok = false;
        } else if (s.compare(i, 4, "true") == 0 || s.compare(i, 4, "null") == 0) {
            i += 4;
        } else if (s.compare(i, 5, "false") == 0) {
            i += 5;
        } else {
            num();
        }
    }
};

bool set_field(framrir_launch& l, const std::string& k, int v) {
    if (k == "lds_bytes") l.lds_bytes = v;
    else if (k == "wg_threads") l.wg_threads = v;
    else if (k == "grid_wgs") l.grid_wgs = v;
    else if (k == "max_mic_group") l.max_mic_group = v;
    else if (k == "waves_per_simd") l.waves_per_simd = v;
    else if (k == "bwd_wg_threads") l.bwd_wg_threads = v;
    else if (k == "bwd_grid_wgs") l.bwd_grid_wgs = v;
    else if (k == "render_path") l.render_path = v;
    else return false;
    return true;
}

// Entries of a cache file; false (and nothing added) when it is missing or
// not in the format.
bool load_cache(const std::string& path, std::map<std::string, Entry>& into) {
    std::ifstream f(path);
    if (!f) return false;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string text = ss.str();
    Json j(text);
    std::map<std::string, Entry> got;
    if (!j.eat('{')) return false;
    if (!j.eat('}')) {
        do {
            const std::string key = j.str();
            if (!j.ok || !j.eat(':') || !j.eat('{')) return false;
            Entry e{default_launch(), 0.0};
            if (!j.eat('}')) {
                do {
                    const std::string field = j.str();
                    if (!j.ok || !j.eat(':')) return false;
                    if (field == "ms") {
                        e.ms = j.num();
                    } else if (field == "launch") {
                        if (!j.eat('{')) return false;
                        if (!j.eat('}')) {
                            do {
                                const std::string name = j.str();
                                if (!j.ok || !j.eat(':')) return false;
                                const double v = j.num();
                                set_field(e.launch, name, static_cast<int>(v));
                            } while (j.ok && j.eat(','));
                            if (!j.eat('}')) return false;
                        }
                    } else {
                        j.skip();
                    }
                } while (j.ok && j.eat(','));
                if (!j.eat('}')) return false;
            }
            if (!j.ok) return false;
            got[key] = e;
        } while (j.eat(','));
        if (!j.eat('}')) return false;
    }
    for (const auto& kv : got) into[kv.first] = kv.second;
    return true;
}

std::string json_escape(const std::string& s) {
    std::string o;
    for (char c : s) {
        if (c == '"' || c == '\\') o.push_back('\\');
        o.push_back(c);
    }
    return o;
}

bool write_cache(const std::string& path, const std::map<std::string, Entry>& entries) {
    const std::string tmp = path + ".tmp";
    {
        std::ofstream f(tmp);
        if (!f) return false;
        f << "{\n";
        size_t n = 0;
        for (const auto& kv : entries) {
            const framrir_launch& l = kv.second.launch;
            char ms[64];
            std::snprintf(ms, sizeof(ms), "%.4f", kv.second.ms);
            f << " \"" << json_escape(kv.first) << "\": {\n  \"launch\": {\n"
              << "   \"bwd_grid_wgs\": " << l.bwd_grid_wgs << ",\n"
              << "   \"bwd_wg_threads\": " << l.bwd_wg_threads << ",\n"
              << "   \"grid_wgs\": " << l.grid_wgs << ",\n"
              << "   \"lds_bytes\": " << l.lds_bytes << ",\n"
              << "   \"max_mic_group\": " << l.max_mic_group << ",\n"
              << "   \"render_path\": " << l.render_path << ",\n"
              << "   \"waves_per_simd\": " << l.waves_per_simd << ",\n"
              << "   \"wg_threads\": " << l.wg_threads << "\n  },\n"
              << "  \"ms\": " << ms << "\n }" << (++n < entries.size() ? "," : "") << "\n";
        }
        f << "}\n";
        if (!f) return false;
    }
    return std::rename(tmp.c_str(), path.c_str()) == 0;
}

// The candidate shapes of the default search: the scatter at several LDS
// tiles, workgroup sizes, register budgets, microphone groups and grid
// sizes, and the bin-moment render at a few tiles.
std::vector<framrir_launch> default_candidates() {
    std::vector<framrir_launch> c;
    const int shapes[][3] = {{131072, 1024, 4}, {98304, 1024, 4}, {65536, 1024, 8}, {49152, 1024, 8},
                             {40960, 1024, 8},  {65536, 512, 4},  {49152, 512, 8},  {40960, 512, 8},
                             {32768, 256, 4}};
    for (const auto& sh : shapes) {
        const int lds = sh[0], t = sh[1], w = sh[2];
        if (lds + framrir::render_static_lds(t) > kLdsPerCu) continue;
        const int per_cu = std::max(1, std::min(kLdsPerCu / (lds + framrir::render_static_lds(t)), w * 4 / (t / 64)));
        for (int g : {8, 4})
            for (int k = 1; k <= per_cu; ++k) c.push_back(framrir_launch{lds, t, 256 * k, g, w, 0, 0, 0});
    }
    const int moments[][3] = {{65536, 512, 2}, {65536, 512, 1}, {49152, 256, 1}, {160000, 1024, 2}};
    for (const auto& m : moments) c.push_back(framrir_launch{m[0], m[1], 0, m[2], 4, 0, 0, 1});
    return c;
}

}  // namespace

struct framrir_handle {
    int device = 0;
    std::string arch;                       // gcnArchName up to the first ':'
    std::string cache_path;                 // written by framrir_tune ("" = memory only)
    std::map<std::string, Entry> entries;   // "arch|class" -> best shape
};

extern "C" int framrir_arch_supported(const char* gcn_arch_name) {
    if (!gcn_arch_name) return 0;
    return std::strncmp(gcn_arch_name, "gfx950", 6) == 0 &&
                   (gcn_arch_name[6] == '\0' || gcn_arch_name[6] == ':')
               ? 1
               : 0;
}

extern "C" int framrir_handle_create(int32_t device, const char* tune_cache_paths, framrir_handle** out) {
    if (!out) return fr_fail(FRAMRIR_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int n_dev = 0;
    hipError_t e = hipGetDeviceCount(&n_dev);
    if (e != hipSuccess) return fr_fail(FRAMRIR_E_DEVICE, "hipGetDeviceCount: %s", hipGetErrorString(e));
    if (device < 0 || device >= n_dev) return fr_fail(FRAMRIR_E_INVALID_ARG, "device %d of %d", device, n_dev);
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return fr_fail(FRAMRIR_E_DEVICE, "hipGetDeviceProperties: %s", hipGetErrorString(e));
    if (!framrir_arch_supported(prop.gcnArchName))
        return fr_fail(FRAMRIR_E_UNSUPPORTED, "device %d is %s; this library is built for gfx950", device,
                       prop.gcnArchName);
    if (int rc = framrir_scratch_setup(device)) return rc;
    framrir_handle* h = new (std::nothrow) framrir_handle();
    if (!h) return fr_fail(FRAMRIR_E_INVALID_ARG, "out of host memory");
    h->device = device;
    h->arch = std::string(prop.gcnArchName).substr(0, std::string(prop.gcnArchName).find(':'));
    // paths separated by ':'; the first is the writable cache, the others
    // read-only fallbacks; the writable one's entries take precedence
    std::vector<std::string> paths;
    if (tune_cache_paths) {
        std::string p(tune_cache_paths);
        size_t b = 0;
        while (b <= p.size()) {
            const size_t c = p.find(':', b);
            paths.push_back(p.substr(b, c == std::string::npos ? std::string::npos : c - b));
            if (c == std::string::npos) break;
            b = c + 1;
        }
    }
    if (!paths.empty()) h->cache_path = paths[0];
    for (size_t k = paths.size(); k-- > 0;)
        if (!paths[k].empty()) load_cache(paths[k], h->entries);
    *out = h;
    return FRAMRIR_OK;
}

extern "C" void framrir_handle_destroy(framrir_handle* h) { delete h; }

extern "C" int framrir_size_class(const framrir_room* rooms, int32_t n_rooms, char* buf, size_t n) {
    if (!rooms || n_rooms <= 0 || !buf || n == 0) return fr_fail(FRAMRIR_E_INVALID_ARG, "rooms and buf required");
    std::vector<int> fs;
    int64_t t_min = INT64_MAX, t_max = 0;
    int mics = 0;
    for (int32_t b = 0; b < n_rooms; ++b) {
        const int64_t T = static_cast<int64_t>(std::ceil(rooms[b].rt60 * rooms[b].fs));
        if (!(T >= 1)) return fr_fail(FRAMRIR_E_RANGE, "room %d: T60 fs < 1", b);
        t_min = std::min(t_min, T);
        t_max = std::max(t_max, T);
        mics = std::max(mics, rooms[b].n_mic);
        const int f = static_cast<int>(rooms[b].fs);
        if (std::find(fs.begin(), fs.end(), f) == fs.end()) fs.push_back(f);
    }
    std::sort(fs.begin(), fs.end());
    int64_t lo = 1, hi = 1;
    while (lo * 2 <= t_min) lo *= 2;
    while (hi < t_max) hi *= 2;
    std::string s = "fs=";
    for (size_t k = 0; k < fs.size(); ++k) s += (k ? "/" : "") + std::to_string(fs[k]);
    s += ";mics<=" + std::to_string(mics) + ";T=" + std::to_string(lo) + "-" + std::to_string(hi);
    std::snprintf(buf, n, "%s", s.c_str());
    return static_cast<int>(s.size()) < static_cast<int>(n) ? FRAMRIR_OK
                                                           : fr_fail(FRAMRIR_E_WORKSPACE, "buf shorter than %zu",
                                                                     s.size() + 1);
}

extern "C" int framrir_tune_lookup(const framrir_handle* h, const char* size_class, framrir_launch* out,
                                   int32_t* found) {
    if (!h || !size_class || !out || !found) return fr_fail(FRAMRIR_E_INVALID_ARG, "NULL argument");
    const auto it = h->entries.find(h->arch + "|" + size_class);
    *found = it != h->entries.end() ? 1 : 0;
    *out = *found ? it->second.launch : default_launch();
    return FRAMRIR_OK;
}

namespace {

// Device buffers of one timed candidate; freed on destruction.
struct DevBuf {
    void* p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    int alloc(size_t n) {
        const hipError_t e = hipMalloc(&p, std::max<size_t>(n, 256));
        return e == hipSuccess ? FRAMRIR_OK : fr_fail(FRAMRIR_E_DEVICE, "hipMalloc(%zu): %s", n, hipGetErrorString(e));
    }
};

// Median time (ms) of framrir_forward for one candidate, or a negative code
// when the shape is not valid for this batch.
int time_candidate(const framrir_room* rooms, int32_t n_rooms, const framrir_params* prm, const double* src,
                   const double* mic, const framrir_launch& l, int reps, hipStream_t st, double* ms) {
    framrir_plan* plan = nullptr;
    int rc = framrir_plan_create(rooms, n_rooms, prm, &l, src, mic, &plan);
    if (rc) return rc;
    struct PlanGuard {
        framrir_plan* p;
        ~PlanGuard() { framrir_plan_destroy(p); }
    } guard{plan};
    framrir_plan_info info;
    if ((rc = framrir_plan_get_info(plan, &info))) return rc;
    DevBuf desc, table, dmic, dsrc, out, ws;
    if ((rc = desc.alloc(info.desc_bytes)) || (rc = table.alloc(32 * info.n_img)) ||
        (rc = dmic.alloc(24 * static_cast<size_t>(info.n_mic))) ||
        (rc = dsrc.alloc(24 * static_cast<size_t>(info.n_src))) || (rc = out.alloc(4 * info.out_floats)) ||
        (rc = ws.alloc(info.ws_bytes)))
        return rc;
    if (hipMemcpyAsync(desc.p, framrir_plan_desc(plan), info.desc_bytes, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(dmic.p, mic, 24 * static_cast<size_t>(info.n_mic), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(dsrc.p, src, 24 * static_cast<size_t>(info.n_src), hipMemcpyHostToDevice, st) != hipSuccess)
        return fr_fail(FRAMRIR_E_DEVICE, "copy of the plan to the device failed");
    if ((rc = framrir_workspace_init(ws.p, info.ws_bytes, st))) return rc;
    auto fwd = [&]() {
        return framrir_forward(plan, desc.p, static_cast<double*>(table.p), static_cast<const double*>(dmic.p),
                               static_cast<const double*>(dsrc.p), nullptr, static_cast<float*>(out.p), ws.p,
                               info.ws_bytes, st);
    };
    for (int k = 0; k < 2; ++k)
        if ((rc = fwd())) return rc;
    std::vector<hipEvent_t> ev(2 * reps);
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) return fr_fail(FRAMRIR_E_DEVICE, "hipEventCreate failed");
    for (int k = 0; k < reps && !rc; ++k) {
        (void)hipEventRecord(ev[2 * k], st);
        rc = fwd();
        (void)hipEventRecord(ev[2 * k + 1], st);
    }
    const hipError_t e = hipStreamSynchronize(st);
    std::vector<double> t;
    for (int k = 0; k < reps && !rc && e == hipSuccess; ++k) {
        float v = 0.0f;
        (void)hipEventElapsedTime(&v, ev[2 * k], ev[2 * k + 1]);
        t.push_back(v);
    }
    for (auto& x : ev) (void)hipEventDestroy(x);
    if (rc) return rc;
    if (e != hipSuccess) return fr_fail(FRAMRIR_E_DEVICE, "tuning run failed: %s", hipGetErrorString(e));
    std::sort(t.begin(), t.end());
    *ms = t[t.size() / 2];
    return FRAMRIR_OK;
}

}  // namespace

extern "C" int framrir_tune(framrir_handle* h, const framrir_room* rooms, int32_t n_rooms, const framrir_params* prm,
                            const double* src, const double* mic, const char* size_class,
                            const framrir_launch* candidates, int32_t n_candidates, int32_t reps,
                            framrir_launch* best, double* best_ms) {
    if (!h || !rooms || !src || !mic || !best) return fr_fail(FRAMRIR_E_INVALID_ARG, "NULL argument");
    if (n_candidates < 0 || (n_candidates > 0 && !candidates) || reps < 1)
        return fr_fail(FRAMRIR_E_INVALID_ARG, "candidates / reps");
    char cls[256];
    if (!size_class) {
        if (int rc = framrir_size_class(rooms, n_rooms, cls, sizeof(cls))) return rc;
        size_class = cls;
    }
    std::vector<framrir_launch> cand = n_candidates > 0
                                           ? std::vector<framrir_launch>(candidates, candidates + n_candidates)
                                           : default_candidates();
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(h->device) != hipSuccess)
        return fr_fail(FRAMRIR_E_DEVICE, "cannot select device %d", h->device);
    hipStream_t st = nullptr;
    if (hipStreamCreate(&st) != hipSuccess) {
        (void)hipSetDevice(prev);
        return fr_fail(FRAMRIR_E_DEVICE, "hipStreamCreate failed");
    }
    double bms = 0.0;
    int found = -1, rc_any = FRAMRIR_OK;
    for (size_t k = 0; k < cand.size(); ++k) {
        double ms = 0.0;
        const int rc = time_candidate(rooms, n_rooms, prm, src, mic, cand[k], reps, st, &ms);
        if (rc == FRAMRIR_E_DEVICE) {   // a device error ends the search
            rc_any = rc;
            break;
        }
        if (rc) continue;   // not a valid shape for this batch
        if (found < 0 || ms < bms) {
            found = static_cast<int>(k);
            bms = ms;
        }
    }
    (void)hipStreamDestroy(st);
    (void)hipSetDevice(prev);
    if (rc_any) return rc_any;
    if (found < 0) return fr_fail(FRAMRIR_E_RANGE, "no candidate launch shape is valid for this batch");
    *best = cand[found];
    if (best_ms) *best_ms = bms;
    const std::string key = h->arch + "|" + size_class;
    h->entries[key] = Entry{cand[found], bms};
    if (!h->cache_path.empty()) {
        std::map<std::string, Entry> own;
        load_cache(h->cache_path, own);   // keep what other runs stored
        own[key] = Entry{cand[found], bms};
        if (!write_cache(h->cache_path, own))
            return fr_fail(FRAMRIR_E_INVALID_ARG, "cannot write the tuning cache %s", h->cache_path.c_str());
    }
    return FRAMRIR_OK;
}
