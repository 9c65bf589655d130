// Schedule tuner of the multi-RHS apply (declared in cstar_internal.h).
//
// A multi-RHS launch of the time-marching kernel can run with several
// schedules (right-hand sides per lane, rows of a workgroup, slices per
// segment) that produce the same result.  The first launch of a kind --
// precision, lattice, number of right-hand sides and epilogue operands --
// times every candidate with HIP events on the caller's stream (one warm-up
// and two timed launches each) and keeps the fastest for the rest of the
// process.  With CSTAR_TUNE_CACHE=<file> the choices are read from and
// appended to that file ("prec T L nrhs operands schedule" per line), so a
// later process skips the measurement; CSTAR_MARCH_SCHEDULE=<n> forces
// schedule n everywhere.  Launches that must not measure (ApplyArgs::no_tune)
// take a choice already made, else schedule 1.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>

#include "cstar_internal.h"

namespace cstar {

namespace {
using Key = std::tuple<int, int, int, int, int>;  // prec, T, L, nrhs, epilogue operands (-1: none)
std::mutex g_mu;
std::map<Key, int> g_table;
bool g_loaded = false;

void load_cache() {
    g_loaded = true;
    const char *path = getenv("CSTAR_TUNE_CACHE");
    if (!path || !path[0]) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    int p, T, L, n, o, sch;
    while (fscanf(f, "%d %d %d %d %d %d", &p, &T, &L, &n, &o, &sch) == 6)
        if (sch >= 0 && sch < kMarchSchedules) g_table[Key(p, T, L, n, o)] = sch;
    fclose(f);
}

void save_entry(const Key &k, int sch) {
    const char *path = getenv("CSTAR_TUNE_CACHE");
    if (!path || !path[0]) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%d %d %d %d %d %d\n", std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k), std::get<4>(k),
            sch);
    fclose(f);
}
}  // namespace

int march_schedule(const Geo &g, cstar_prec prec, const ApplyArgs &a, hipStream_t s,
                   const std::function<void(int)> &launch) {
    if (const char *f = getenv("CSTAR_MARCH_SCHEDULE")) {
        const int v = atoi(f);
        if (v >= 0 && v < kMarchSchedules) return v;
    }
    const bool epi = a.y || a.z || a.w || a.ea != 1.0;
    const int ops = epi ? (a.y ? 1 : 0) + (a.z ? 1 : 0) + (a.w ? 1 : 0) : -1;
    const Key key((int)prec, g.T, g.L, a.nrhs, ops);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_loaded) load_cache();
    auto it = g_table.find(key);
    if (it != g_table.end()) return it->second;
    if (a.no_tune) return 1;  // two right-hand sides per lane, 2 x 4 rows, 8 slices
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return 0;
    }
    float t[kMarchSchedules];
    float best_ms = 1e30f;
    for (int sch = 0; sch < kMarchSchedules; sch++) {
        launch(sch);
        (void)hipEventRecord(e0, s);
        launch(sch);
        launch(sch);
        (void)hipEventRecord(e1, s);
        float ms = 1e30f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) ms = 1e30f;
        t[sch] = ms;
        best_ms = std::min(best_ms, ms);
    }
    // the lowest-numbered schedule within 2 % of the fastest: timing noise
    // between near-equal schedules does not change the choice from run to run
    int best = 0;
    while (best + 1 < kMarchSchedules && !(t[best] <= 1.02f * best_ms)) best++;
    best_ms = t[best];
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (getenv("CSTAR_VERBOSE"))
        fprintf(stderr, "[cstar tune] prec %d %dx%d^3 nrhs %d operands %d: schedule %d (%.3f ms per launch)\n", (int)prec,
                g.T, g.L, a.nrhs, ops, best, best_ms / 2);
    g_table[key] = best;
    save_entry(key, best);
    return best;
}

}  // namespace cstar
