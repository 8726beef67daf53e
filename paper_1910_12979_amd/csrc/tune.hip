// Fused-sweep tuning table and its persistent JSON cache.
//
// The autotuner (mg_autotune) times every tile configuration on each level
// shape of a hierarchy and records the fastest here, keyed by the GPU
// architecture (the device's gcnArchName, e.g. "gfx950:sramecc+:xnack-"),
// the level shape, the coefficient source (rho or stored), the precision and
// whether the level is a coarse level.  With the environment variable
// MACPROJ_TUNE_CACHE naming a file, the table is read from that file the
// first time it is consulted and written back (whole, replacing the file
// atomically) after every mg_autotune, so later processes start tuned.
//
// File format (written and read by this module only):
//   {"format": "macproj-sweep-tune-1",
//    "entries": [
//      {"arch": "gfx950:sramecc+:xnack-", "n": [256, 256, 256], "rho": 1,
//       "fp64": 1, "coarse": 0, "cfg": 11, "tile": [64, 16, 64]},
//      ...]}
// An entry whose "tile" does not match the configuration index in this
// build, or whose fields are missing or out of range, is skipped.
#include <hip/hip_runtime.h>

#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include <unistd.h>

#include "mg_internal.h"
#include "runtime.h"
#include "sweep.h"

namespace mg {
namespace {

using TuneKey = std::tuple<std::string, int, int, int, int, int, int>;   // arch, nx, ny, nz, rho, fp64, coarse

std::mutex g_mu;
std::map<TuneKey, int> g_table;
int g_forced = -1;
unsigned g_epoch = 0;
bool g_env_loaded = false;
std::map<int, std::string> g_arch;          // device -> architecture name

const char* kFormat = "macproj-sweep-tune-1";

std::string current_arch() {
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess) return "unknown";
    auto it = g_arch.find(d);
    if (it != g_arch.end()) return it->second;
    hipDeviceProp_t prop;
    std::string a = "unknown";
    if (hipGetDeviceProperties(&prop, d) == hipSuccess) a = prop.gcnArchName;
    g_arch[d] = a;
    return a;
}

// ---- a small reader for the file format above --------------------------------
struct Reader {
    const std::string& s;
    size_t i = 0;
    explicit Reader(const std::string& t) : s(t) {}
    void ws() {
        while (i < s.size() && std::isspace((unsigned char)s[i])) ++i;
    }
    bool eat(char c) {
        ws();
        if (i < s.size() && s[i] == c) {
            ++i;
            return true;
        }
        return false;
    }
    bool str(std::string& out) {
        ws();
        if (i >= s.size() || s[i] != '"') return false;
        ++i;
        out.clear();
        while (i < s.size() && s[i] != '"') {
            if (s[i] == '\\' && i + 1 < s.size()) ++i;
            out.push_back(s[i++]);
        }
        if (i >= s.size()) return false;
        ++i;
        return true;
    }
    bool num(long long& v) {
        ws();
        size_t j = i;
        if (j < s.size() && (s[j] == '-' || s[j] == '+')) ++j;
        size_t d0 = j;
        while (j < s.size() && std::isdigit((unsigned char)s[j])) ++j;
        if (j == d0 || j - d0 > 12) return false;
        v = std::strtoll(s.substr(i, j - i).c_str(), nullptr, 10);
        i = j;
        return true;
    }
    // skip any value (used for unknown keys)
    bool skip() {
        ws();
        if (i >= s.size()) return false;
        if (s[i] == '"') {
            std::string t;
            return str(t);
        }
        if (s[i] == '[' || s[i] == '{') {
            const char open = s[i], close = open == '[' ? ']' : '}';
            int depth = 0;
            for (; i < s.size(); ++i) {
                if (s[i] == '"') {
                    std::string t;
                    if (!str(t)) return false;
                    --i;
                    continue;
                }
                if (s[i] == open) ++depth;
                if (s[i] == close && --depth == 0) {
                    ++i;
                    return true;
                }
            }
            return false;
        }
        long long v;
        if (num(v)) return true;
        for (const char* w : {"true", "false", "null"})
            if (s.compare(i, std::strlen(w), w) == 0) {
                i += std::strlen(w);
                return true;
            }
        return false;
    }
    bool ints(std::vector<long long>& out) {
        out.clear();
        if (!eat('[')) return false;
        if (eat(']')) return true;
        for (;;) {
            long long v;
            if (!num(v)) return false;
            out.push_back(v);
            if (eat(']')) return true;
            if (!eat(',')) return false;
        }
    }
};

struct Entry {
    std::string arch;
    std::vector<long long> n, tile;
    long long rho = -1, fp64 = -1, coarse = -1, cfg = -1;
};

bool read_entry(Reader& r, Entry& e) {
    if (!r.eat('{')) return false;
    if (r.eat('}')) return true;
    for (;;) {
        std::string k;
        if (!r.str(k) || !r.eat(':')) return false;
        bool ok;
        if (k == "arch") ok = r.str(e.arch);
        else if (k == "n") ok = r.ints(e.n);
        else if (k == "tile") ok = r.ints(e.tile);
        else if (k == "rho") ok = r.num(e.rho);
        else if (k == "fp64") ok = r.num(e.fp64);
        else if (k == "coarse") ok = r.num(e.coarse);
        else if (k == "cfg") ok = r.num(e.cfg);
        else ok = r.skip();
        if (!ok) return false;
        if (r.eat('}')) return true;
        if (!r.eat(',')) return false;
    }
}

bool entry_valid(const Entry& e) {
    if (e.arch.empty() || e.n.size() != 3 || e.cfg < 0 || e.cfg >= kNumSweepCfg) return false;
    for (long long v : e.n)
        if (v < 1 || v > (1 << 20)) return false;
    if ((e.rho != 0 && e.rho != 1) || (e.fp64 != 0 && e.fp64 != 1) || (e.coarse != 0 && e.coarse != 1)) return false;
    const SweepCfg& c = kSweepCfgs[e.cfg];
    if (e.tile.size() != 3 || e.tile[0] != c.tx || e.tile[1] != c.ty || e.tile[2] != c.tz) return false;
    return sweep_cfg_fits((int)e.n[0], (int)e.n[1], (int)e.cfg);
}

// Merge the file's valid entries into the table (caller holds g_mu).  Returns
// the entries taken, or MG_ERR_INVALID_ARG if the file cannot be read or is
// not a cache file.
int load_locked(const char* path) {
    FILE* fp = std::fopen(path, "rb");
    if (!fp) {
        set_error(std::string("cannot open tuning cache ") + path);
        return MG_ERR_INVALID_ARG;
    }
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof buf, fp)) > 0 && text.size() < ((size_t)64 << 20)) text.append(buf, got);
    std::fclose(fp);
    Reader r(text);
    if (!r.eat('{')) {
        set_error("tuning cache is not a JSON object");
        return MG_ERR_INVALID_ARG;
    }
    bool format_ok = false;
    std::vector<Entry> entries;
    if (!r.eat('}')) {
        for (;;) {
            std::string k;
            if (!r.str(k) || !r.eat(':')) {
                set_error("malformed tuning cache");
                return MG_ERR_INVALID_ARG;
            }
            bool ok;
            if (k == "format") {
                std::string f;
                ok = r.str(f);
                format_ok = ok && f == kFormat;
            } else if (k == "entries") {
                ok = r.eat('[');
                if (ok && !r.eat(']')) {
                    for (;;) {
                        Entry e;
                        if (!read_entry(r, e)) {
                            ok = false;
                            break;
                        }
                        entries.push_back(e);
                        if (r.eat(']')) break;
                        if (!r.eat(',')) {
                            ok = false;
                            break;
                        }
                    }
                }
            } else {
                ok = r.skip();
            }
            if (!ok) {
                set_error("malformed tuning cache");
                return MG_ERR_INVALID_ARG;
            }
            if (r.eat('}')) break;
            if (!r.eat(',')) {
                set_error("malformed tuning cache");
                return MG_ERR_INVALID_ARG;
            }
        }
    }
    if (!format_ok) {
        set_error(std::string("tuning cache format is not ") + kFormat);
        return MG_ERR_INVALID_ARG;
    }
    int taken = 0;
    for (const Entry& e : entries) {
        if (!entry_valid(e)) continue;
        g_table[TuneKey(e.arch, (int)e.n[0], (int)e.n[1], (int)e.n[2], (int)e.rho, (int)e.fp64, (int)e.coarse)] =
            (int)e.cfg;
        ++taken;
    }
    ++g_epoch;
    return taken;
}

std::string json_escape(const std::string& s) {
    std::string o;
    for (char c : s) {
        if (c == '"' || c == '\\') o.push_back('\\');
        if ((unsigned char)c >= 0x20) o.push_back(c);
    }
    return o;
}

// Write the whole table to path (caller holds g_mu): a temporary file
// renamed over the target, so readers never see half a file.
int save_locked(const char* path) {
    static unsigned serial = 0;
    const std::string tmp = std::string(path) + ".tmp" + std::to_string((long long)getpid()) + "." +
                            std::to_string(++serial);
    FILE* fp = std::fopen(tmp.c_str(), "wb");
    if (!fp) {
        set_error(std::string("cannot write tuning cache ") + path);
        return MG_ERR_INVALID_ARG;
    }
    std::fprintf(fp, "{\"format\": \"%s\",\n \"entries\": [", kFormat);
    int n = 0;
    for (const auto& kv : g_table) {
        const TuneKey& k = kv.first;
        const SweepCfg& c = kSweepCfgs[kv.second];
        std::fprintf(fp,
                     "%s\n  {\"arch\": \"%s\", \"n\": [%d, %d, %d], \"rho\": %d, \"fp64\": %d, \"coarse\": %d, "
                     "\"cfg\": %d, \"tile\": [%d, %d, %d]}",
                     n ? "," : "", json_escape(std::get<0>(k)).c_str(), std::get<1>(k), std::get<2>(k), std::get<3>(k),
                     std::get<4>(k), std::get<5>(k), std::get<6>(k), kv.second, c.tx, c.ty, c.tz);
        ++n;
    }
    std::fprintf(fp, "\n ]}\n");
    const bool ok = std::fflush(fp) == 0;
    std::fclose(fp);
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        set_error(std::string("cannot replace tuning cache ") + path);
        return MG_ERR_INVALID_ARG;
    }
    return n;
}

const char* env_path() {
    const char* p = std::getenv("MACPROJ_TUNE_CACHE");
    return (p && *p) ? p : nullptr;
}

// The cache file named by the environment, read once (caller holds g_mu);
// a missing file is an empty cache.
void env_load_locked() {
    if (g_env_loaded) return;
    g_env_loaded = true;
    const char* p = env_path();
    if (!p) return;
    FILE* fp = std::fopen(p, "rb");
    if (!fp) return;
    std::fclose(fp);
    (void)load_locked(p);
}

}  // namespace

int tune_find(int nx, int ny, int nz, bool rho, bool dbl, bool coarse) {
    std::lock_guard<std::mutex> lk(g_mu);
    env_load_locked();
    auto it = g_table.find(TuneKey(current_arch(), nx, ny, nz, rho ? 1 : 0, dbl ? 1 : 0, coarse ? 1 : 0));
    return it == g_table.end() ? -1 : it->second;
}

void tune_put(int nx, int ny, int nz, bool rho, bool dbl, bool coarse, int cfg) {
    std::lock_guard<std::mutex> lk(g_mu);
    env_load_locked();
    g_table[TuneKey(current_arch(), nx, ny, nz, rho ? 1 : 0, dbl ? 1 : 0, coarse ? 1 : 0)] = cfg;
    ++g_epoch;
}

int tune_count() {
    std::lock_guard<std::mutex> lk(g_mu);
    return (int)g_table.size();
}

unsigned tune_epoch() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_epoch;
}

void tune_force(int cfg) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_forced = cfg;
    ++g_epoch;
}

int tune_forced() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_forced;
}

int tune_save_env() {
    const char* p = env_path();
    if (!p) return 0;
    std::lock_guard<std::mutex> lk(g_mu);
    return save_locked(p);
}

}  // namespace mg

using namespace mg;

extern "C" {

int mg_tune_cache_save(const char* path) {
    try {
        const char* p = path ? path : env_path();
        if (!p) {
            set_error("no path given and MACPROJ_TUNE_CACHE is not set");
            return MG_ERR_INVALID_ARG;
        }
        std::lock_guard<std::mutex> lk(g_mu);
        env_load_locked();
        return save_locked(p);
    } catch (...) {
        set_error("internal error in mg_tune_cache_save");
        return MG_ERR_HIP;
    }
}

int mg_tune_cache_load(const char* path) {
    try {
        const char* p = path ? path : env_path();
        if (!p) {
            set_error("no path given and MACPROJ_TUNE_CACHE is not set");
            return MG_ERR_INVALID_ARG;
        }
        std::lock_guard<std::mutex> lk(g_mu);
        g_env_loaded = true;             // an explicit load replaces the lazy one
        return load_locked(p);
    } catch (...) {
        set_error("internal error in mg_tune_cache_load");
        return MG_ERR_HIP;
    }
}

int mg_tune_cache_clear(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_table.clear();
    g_env_loaded = true;                 // do not re-read the environment's file
    ++g_epoch;
    return MG_OK;
}

int mg_tune_record(const char* arch, const int32_t n[3], int32_t rho, int32_t fp64, int32_t coarse, int32_t cfg) {
    if (!n || cfg < 0 || cfg >= kNumSweepCfg || n[0] < 1 || n[1] < 1 || n[2] < 1 || !sweep_cfg_fits(n[0], n[1], cfg)) {
        set_error("bad tuning entry");
        return MG_ERR_INVALID_ARG;
    }
    try {
        std::lock_guard<std::mutex> lk(g_mu);
        env_load_locked();
        const std::string a = arch ? std::string(arch) : current_arch();
        g_table[TuneKey(a, n[0], n[1], n[2], rho ? 1 : 0, fp64 ? 1 : 0, coarse ? 1 : 0)] = cfg;
        ++g_epoch;
        return MG_OK;
    } catch (...) {
        set_error("internal error in mg_tune_record");
        return MG_ERR_HIP;
    }
}

int mg_tune_lookup(const char* arch, const int32_t n[3], int32_t rho, int32_t fp64, int32_t coarse) {
    if (!n) return -1;
    try {
        std::lock_guard<std::mutex> lk(g_mu);
        env_load_locked();
        const std::string a = arch ? std::string(arch) : current_arch();
        auto it = g_table.find(TuneKey(a, n[0], n[1], n[2], rho ? 1 : 0, fp64 ? 1 : 0, coarse ? 1 : 0));
        return it == g_table.end() ? -1 : it->second;
    } catch (...) {
        return -1;
    }
}

}  // extern "C"
