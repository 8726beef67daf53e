// Host-side checks of the library's C ABI under AddressSanitizer and
// UndefinedBehaviorSanitizer (built host-only by tests/test_host_sanitize.py;
// no device code, no GPU): parameter validation over random and extreme
// inputs, null-handle and bad-argument paths, status strings, and the
// tuning-cache reader fed with valid, truncated and corrupted files.  Every
// call here must return a status without touching a device.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <random>
#include <string>

#include "macproj.h"

static int g_fail = 0;
#define CHECK(cond)                                                           \
    do {                                                                      \
        if (!(cond)) {                                                        \
            std::fprintf(stderr, "check failed (line %d): %s\n", __LINE__, #cond); \
            ++g_fail;                                                         \
        }                                                                     \
    } while (0)

static void fuzz_params(std::mt19937& rng) {
    const double specials[] = {0.0, -1.0, 1e-300, 1e300, std::numeric_limits<double>::infinity(),
                               std::numeric_limits<double>::quiet_NaN(), 1.0 / 64, 1.0};
    std::uniform_int_distribution<int> dim(-3, 700), bc(-2, 7), sw(-2, 5), prec(-1, 3), cyc(-5, 200000), pick(0, 7);
    for (int it = 0; it < 20000; ++it) {
        mg_params p;
        mg_default_params(&p, dim(rng), dim(rng), dim(rng), specials[pick(rng)]);
        if (it % 3) {
            for (int d = 0; d < 3; ++d) p.bc[d] = bc(rng);
            p.pre_sweeps = sw(rng);
            p.post_sweeps = sw(rng);
            p.precision = prec(rng);
            p.max_cycles = cyc(rng);
            p.rtol = specials[pick(rng)];
            p.inner_cycles = sw(rng) * 3;
        }
        const int levels = mg_num_levels_for(&p);
        const size_t bytes = mg_workspace_bytes(&p);
        CHECK(levels >= 0 && levels <= 24);
        if (levels == 0) CHECK(bytes == 0);
        const int nl = nodal_num_levels_for(&p);
        CHECK(nl >= 0 && nl <= 24);
    }
    // shapes that coarsen to a solvable level and ones that do not
    mg_params p;
    mg_default_params(&p, 256, 256, 256, 1.0 / 256);
    CHECK(mg_num_levels_for(&p) == 7 && mg_workspace_bytes(&p) > 0);
    mg_default_params(&p, 37, 37, 37, 1.0 / 37);
    CHECK(mg_num_levels_for(&p) == 0 && mg_workspace_bytes(&p) == 0);
    mg_default_params(&p, 1, 1, 1, 1.0);
    CHECK(mg_num_levels_for(&p) == 1);
    CHECK(mg_num_levels_for(nullptr) == 0 && mg_workspace_bytes(nullptr) == 0);
}

static void null_paths() {
    mg_params p;
    mg_default_params(&p, 32, 32, 32, 1.0 / 32);
    mg_stats st;
    double d = 0.0;
    CHECK(mg_destroy(nullptr) == MG_OK);
    CHECK(mg_set_params(nullptr, &p) == MG_ERR_INVALID_ARG);
    CHECK(mg_set_coefficients(nullptr, &d, &d, &d, nullptr) == MG_ERR_INVALID_ARG);
    CHECK(mac_project(nullptr, &d, &d, &d, &d, &d, &d, &d, &d, &st, nullptr) == MG_ERR_INVALID_ARG);
    CHECK(mg_vcycle(nullptr, &d, &d, nullptr, nullptr) == MG_ERR_INVALID_ARG);
    CHECK(mg_setup(&p, nullptr, 0, nullptr) == MG_ERR_INVALID_ARG);
    CHECK(mg_set_graphs(nullptr, 1) == MG_ERR_INVALID_ARG);
    CHECK(mg_set_bottom(nullptr, 1) == MG_ERR_INVALID_ARG);
    CHECK(mg_tune_sweep(99) == MG_ERR_INVALID_ARG && mg_tune_sweep(-2) == MG_ERR_INVALID_ARG);
    CHECK(nodal_tune_sweep(99) == MG_ERR_INVALID_ARG);
    CHECK(nodal_destroy(nullptr) == MG_OK);
    CHECK(project_batch(-1, nullptr, nullptr, nullptr) == MG_ERR_INVALID_ARG);
    CHECK(project_batch(3, nullptr, nullptr, nullptr) == MG_ERR_INVALID_ARG);
    CHECK(project_batch(0, nullptr, nullptr, nullptr) == MG_OK);
    void* srv = nullptr;
    CHECK(serve_create(1 << 20, 0, &srv) == MG_ERR_INVALID_ARG);
    CHECK(serve_create(1 << 20, 4, nullptr) == MG_ERR_INVALID_ARG);
    uint64_t t = 0;
    CHECK(serve_submit(nullptr, nullptr, &t) == MG_ERR_INVALID_ARG);
    CHECK(serve_poll(nullptr, 1, &st) == MG_ERR_INVALID_ARG);
    CHECK(serve_wait(nullptr, 1, &st) == MG_ERR_INVALID_ARG);
    double c[6];
    CHECK(serve_counters(nullptr, c) == MG_ERR_INVALID_ARG);
    CHECK(serve_destroy(nullptr) == MG_OK);
    CHECK(mg_beta0_from_p0(0, 1.0, &d, &d, &d, &d, &d, nullptr) == MG_ERR_INVALID_ARG);
    CHECK(mg_beta0_from_p0(8, -1.0, &d, &d, &d, &d, &d, nullptr) == MG_ERR_INVALID_ARG);
    // the allocation-free entry point rejects bad params before any device call
    mg_params bad = p;
    bad.dx = -1.0;
    CHECK(mac_project_static(&bad, &d, &d, &d, &d, &d, &d, &d, &d, &st, nullptr) == MG_ERR_INVALID_ARG);
    for (int inner : {-1, 9}) {           // FP32 V-cycles per refinement step: 0..8
        bad = p;
        bad.inner_cycles = inner;
        CHECK(mac_project_static(&bad, &d, &d, &d, &d, &d, &d, &d, &d, &st, nullptr) == MG_ERR_INVALID_ARG);
    }
    mg_default_params(&bad, 37, 37, 37, 1.0);
    CHECK(mac_project_static(&bad, &d, &d, &d, &d, &d, &d, &d, &d, &st, nullptr) == MG_ERR_BAD_SIZE);
    for (int code = -20; code <= 5; ++code) CHECK(mg_strerror(code) != nullptr && std::strlen(mg_strerror(code)) > 0);
    CHECK(mg_last_error() != nullptr);
}

static void tune_cache(std::mt19937& rng, const std::string& dir) {
    const char* arch = "gfx950:sanitize";
    mg_tune_cache_clear();
    std::uniform_int_distribution<int> dim(1, 600), cfg(-3, 20), bit(0, 1);
    int recorded = 0;
    for (int it = 0; it < 3000; ++it) {
        const int32_t n[3] = {dim(rng), dim(rng), dim(rng)};
        const int c = cfg(rng);
        const int rc = mg_tune_record(arch, n, bit(rng), bit(rng), bit(rng), c);
        if (rc == MG_OK) ++recorded;
        CHECK(rc == MG_OK || rc == MG_ERR_INVALID_ARG);
        (void)mg_tune_lookup(arch, n, 1, 1, 0);
    }
    CHECK(recorded > 0);
    const std::string path = dir + "/tune.json";
    const int saved = mg_tune_cache_save(path.c_str());
    CHECK(saved > 0);
    mg_tune_cache_clear();
    CHECK(mg_tune_cache_load(path.c_str()) == saved);
    // the file, truncated and corrupted: never a crash, a malformed file changes nothing
    std::string text;
    if (FILE* f = std::fopen(path.c_str(), "rb")) {
        char buf[4096];
        size_t got;
        while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
        std::fclose(f);
    }
    CHECK(!text.empty());
    std::uniform_int_distribution<size_t> pos(0, text.size() - 1);
    std::uniform_int_distribution<int> ch(0, 255), op(0, 3);
    const std::string bad = dir + "/bad.json";
    for (int it = 0; it < 1500; ++it) {
        std::string t = text;
        switch (op(rng)) {
            case 0: t.resize(pos(rng)); break;
            case 1: for (int k = 0; k < 4; ++k) t[pos(rng)] = (char)ch(rng); break;
            case 2: t.erase(pos(rng), 1 + pos(rng) % 64); break;
            default: t.insert(pos(rng), std::string(1 + ch(rng) % 8, "{}[],:\"0\\"[ch(rng) % 9])); break;
        }
        if (FILE* f = std::fopen(bad.c_str(), "wb")) {
            std::fwrite(t.data(), 1, t.size(), f);
            std::fclose(f);
        }
        const int rc = mg_tune_cache_load(bad.c_str());
        CHECK(rc >= 0 || rc == MG_ERR_INVALID_ARG);
    }
    CHECK(mg_tune_cache_load((dir + "/missing.json").c_str()) == MG_ERR_INVALID_ARG);
    CHECK(mg_tune_cache_save((dir + "/no/such/dir/t.json").c_str()) == MG_ERR_INVALID_ARG);
    CHECK(mg_tune_lookup(arch, nullptr, 1, 1, 0) == -1);
    mg_tune_cache_clear();
}

int main(int argc, char** argv) {
    const std::string dir = argc > 1 ? argv[1] : ".";
    std::mt19937 rng(12345);
    fuzz_params(rng);
    null_paths();
    tune_cache(rng, dir);
    if (g_fail) {
        std::fprintf(stderr, "%d host checks failed\n", g_fail);
        return 1;
    }
    std::printf("host checks passed\n");
    return 0;
}
