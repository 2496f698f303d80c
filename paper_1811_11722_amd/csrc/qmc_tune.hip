// Autotuner for the lattice kernel's launch shape.
//
// For a (plan, integrand) pair it times every compiled shift tile (and, for
// sector integrands, every specialised tile) against a range of grid sizes on
// the device, keeps the fastest, stores it in the plan and records it under a
// key (architecture, family, transform, d, m, floor(log2 n), specialised or
// not) in the cache file named by QMC_TUNE_CACHE.  Plans without an explicit
// launch shape look that cache up before falling back to the defaults.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <mutex>
#include <sstream>

#include "qmc_runtime.hpp"

namespace qmc {

namespace {

std::mutex g_tune_mu;
std::map<std::string, qmc_launch> g_tune;
bool g_tune_loaded = false;

std::string arch_name(int dev) {
    static std::map<int, std::string> cache;
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    hipDeviceProp_t prop;
    std::string a = "unknown";
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        a = prop.gcnArchName;
        a = a.substr(0, a.find(':'));
    }
    cache[dev] = a;
    return a;
}

void load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = std::getenv("QMC_TUNE_CACHE");
    if (!path) return;
    std::ifstream f(path);
    std::string key;
    uint32_t T, b;
    while (f >> key >> T >> b) g_tune[key] = qmc_launch{T, b};
}

}  // namespace

std::string tune_key(const qmc_plan_s *p, const Packed &pk, bool jit) {
    std::ostringstream s;
    s << arch_name(p->device) << "|f" << pk.key_family << "|t" << p->tr.kind << "|a" << p->tr.alpha << "|d" << p->d
      << "|m" << p->m << "|n" << (int)std::floor(std::log2((double)p->n)) << "|j" << (jit ? 1 : 0)
      << (pk.deform ? "|def" : "") << (pk.orders >= 2 ? "|o" + std::to_string(pk.orders) : std::string());
    return s.str();
}

bool tune_lookup(const qmc_plan_s *p, const Packed &pk, bool jit, qmc_launch &out) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    load_locked();
    auto it = g_tune.find(tune_key(p, pk, jit));
    if (it == g_tune.end()) return false;
    out = it->second;
    return true;
}

static void tune_store(const std::string &key, const qmc_launch &l) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    load_locked();
    g_tune[key] = l;
    if (const char *path = std::getenv("QMC_TUNE_CACHE")) {
        std::ofstream f(path, std::ios::app);
        f << key << " " << l.shift_tile << " " << l.blocks_per_cu << "\n";
    }
}

}  // namespace qmc

using namespace qmc;

extern "C" qmc_status qmc_autotune(qmc_plan_t p, qmc_family family, const void *params, qmc_launch *best) {
    if (!p) return fail(QMC_EINVAL, "plan is NULL");
    Packed pk;
    qmc_status st = pack_params((int)family, p->d, params, pk);
    if (st) return st;
    const bool sector = pk.key_family == QMC_F_SECTOR || pk.key_family == kFamSectorComplex;
    const bool jit = sector && p->jit_mode != 0;
    std::vector<uint32_t> tiles;
    for (uint32_t T : {1u, 2u, 4u, 8u}) {
        if (jit) {
            if (T <= 4) tiles.push_back(T);
            continue;
        }
        uint32_t got = 0;
        if (find_kernel(pk.key_family, p->tr, p->d, T, got) && got == T) tiles.push_back(T);
    }
    const qmc_launch keep = p->launch;
    const bool keep_timing = p->timing;
    p->timing = true;
    double best_ms = INFINITY;
    qmc_launch choice{0, 0};
    qmc_result r;
    for (uint32_t T : tiles) {
        for (uint32_t bpc : {2u, 4u, 8u, 16u, 32u}) {
            if ((st = plan_enqueue(p, pk, T, bpc)) || (st = plan_collect(p, pk.np, &r, nullptr))) {
                if (st == QMC_ENONFINITE) continue;
                p->timing = keep_timing;
                return st;
            }
            p->kernel_ms = 0.0;
            p->kernel_launches = 0;
            for (int rep = 0; rep < 3; ++rep)
                if ((st = plan_enqueue(p, pk, T, bpc)) || (st = plan_collect(p, pk.np, &r, nullptr))) break;
            const double ms = p->kernel_launches ? p->kernel_ms / (double)p->kernel_launches : INFINITY;
            if (p->last_T == T && ms < best_ms) {
                best_ms = ms;
                choice = qmc_launch{T, bpc};
            }
        }
    }
    p->timing = keep_timing;
    p->kernel_ms = 0.0;
    p->kernel_launches = 0;
    if (choice.shift_tile == 0) {
        p->launch = keep;
        return fail(QMC_EUNSUPPORTED, "no launch shape ran");
    }
    p->launch = choice;
    tune_store(tune_key(p, pk, jit), choice);
    if (best) *best = choice;
    return QMC_OK;
}
