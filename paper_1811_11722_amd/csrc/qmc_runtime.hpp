// Host-side runtime shared by the C ABI, the batch driver and the autotuner.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/qmc.h"
#include "qmc_registry.hpp"

namespace qmc {

constexpr uint32_t kMaxDim = 16;
constexpr uint32_t kMaxSumSectors = 32;  // sectors in one summed kernel (qmc_integrate_sum)
// Per-plan result buffer: Q_k for up to kMaxParts parts (m * kMaxParts
// doubles), then the results of every pair of parts, (mean a, mean b,
// err a, err b), 4 doubles per pair (kMaxParts in qmc_kernels.hpp).
inline size_t out_res_offset(uint32_t m) { return (size_t)kMaxParts * m; }
inline size_t out_doubles(uint32_t m) { return (size_t)kMaxParts * m + 2 * kMaxParts; }
constexpr uint32_t kMaxTile = 8;  // largest shift tile of any kernel

struct qmc_plan_extra;  // batch / graph state, owned by qmc_batch.hip

}  // namespace qmc

struct qmc_plan_s {
    uint32_t d = 0, n = 0, m = 0;
    double inv_n = 0.0;
    qmc_transform tr{0, 0};
    std::vector<uint32_t> g;
    std::vector<double> shifts;
    int device = 0;
    hipStream_t stream = nullptr;
    // device memory
    uint32_t *d_g = nullptr;
    uint32_t *d_gstep = nullptr;
    double *d_shifts = nullptr;
    double *d_params = nullptr;
    size_t params_cap = 0;  // in doubles
    double2 *d_partials = nullptr;
    size_t partials_cap = 0;  // in bytes
    double *d_out = nullptr;  // q (2m) then res (4)
    double *h_out = nullptr;  // pinned mirror of d_out
    std::vector<double> last_blob;
    uint32_t cur_S = 0;  // thread stride that d_gstep was computed for
    qmc_launch launch{0, 0};
    uint32_t last_T = 0, last_bx = 0;
    int32_t jit_mode = 1;   // 0 tables only, 1 specialise when possible, 2 always specialise
    bool last_jit = false;  // the last sector estimate ran a specialised kernel
    // timing
    bool timing = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double kernel_ms = 0.0;
    uint64_t kernel_launches = 0;
    qmc::qmc_plan_extra *extra = nullptr;
};

namespace qmc {

struct Packed {
    std::vector<double> blob;
    uint32_t np = 1;       // parts accumulated per shift
    int key_family = 0;
    bool cplx = false;     // complex sector
    uint32_t orders = 0;   // expansion orders (>= 2: qmc_integrate_orders)
    bool deform = false;   // contour deformation (complex result, specialised kernel only)
    bool crossing = false; // last part: 1 where the deformed contour has Im(F - i delta) > 0
};

qmc_status fail(qmc_status s, const char *fmt, ...);
qmc_status hip_fail(hipError_t e, const char *what);
int device_cu_count(int dev);
qmc_status pack_params(int family, uint32_t d, const void *params, Packed &pk);
qmc_status validate_rule(uint32_t d, uint64_t n, const uint64_t *g, uint32_t m, const double *shifts,
                         qmc_transform &t);
// order in which the specialised sector code reads a polynomial's terms
std::vector<uint32_t> horner_term_order(const std::vector<uint64_t> &codes, uint32_t d);
double transform_scale(const qmc_transform &t, uint32_t d);
LatticeLaunch find_kernel(int key_family, const qmc_transform &t, uint32_t d, uint32_t want_T, uint32_t &T_out);
uint32_t default_tile(int key_family);
uint32_t grid_x(uint32_t n, uint32_t tiles_total, int dev, uint32_t blocks_per_cu);
void gstep_for(const uint32_t *g, uint32_t d, uint32_t n, uint64_t S, uint32_t *out);
qmc_status ensure_buffer(void **ptr, size_t &cap, size_t bytes, const char *what);
qmc_status plan_upload_params(qmc_plan_s *p, const Packed &pk);
qmc_status plan_set_gstep(qmc_plan_s *p, uint32_t S);
qmc_status plan_enqueue(qmc_plan_s *p, const Packed &pk, uint32_t want_T, uint32_t blocks_per_cu);
qmc_status plan_collect(qmc_plan_s *p, uint32_t np, qmc_result *out, double *per_shift, bool crossing = false);
qmc_status plan_results(qmc_plan_s *p, uint32_t np, qmc_result *out, double *per_shift, bool crossing);
void plan_release_extra(qmc_plan_s *p);
uint32_t padded_rows(uint32_t m);
std::vector<double> padded_shifts(const std::vector<double> &sh, uint32_t m, uint32_t d, uint32_t rows,
                                  const qmc_transform &tr);
hipFunction_t jit_kernel(const std::vector<double> &blob, uint32_t d, const qmc_transform &tr, uint32_t T,
                         bool cplx, int dev, std::string &err);
hipFunction_t jit_sum_kernel(const std::vector<double> &blob, const std::vector<size_t> &offs, uint32_t d,
                             const qmc_transform &tr, uint32_t T, bool cplx, int dev, std::string &err);
hipError_t jit_launch(hipFunction_t fn, const LatticeArgs &a, dim3 grid, hipStream_t s);
struct CvSampleArgs;
hipFunction_t jit_cv_kernel(const std::vector<double> &blob, size_t cv_off, uint32_t d, const qmc_transform &tr,
                            uint32_t R, uint32_t K, bool cplx, int dev, std::string &err);
hipFunction_t jit_sample_kernel(const std::vector<double> &blob, uint32_t d, const qmc_transform &tr, bool cplx, int dev,
                                std::string &err);
hipError_t jit_launch_sample(hipFunction_t fn, const CvSampleArgs &a, uint32_t blocks, hipStream_t s);
qmc_status plan_enqueue_fn(qmc_plan_s *p, const Packed &pk, hipFunction_t jfn, uint32_t T);
std::string tune_key(const qmc_plan_s *p, const Packed &pk, bool jit);
bool tune_lookup(const qmc_plan_s *p, const Packed &pk, bool jit, qmc_launch &out);

// device allocations released together when the object goes out of scope
struct DeviceScratch {
    std::vector<void *> ptr;
    qmc_status alloc(size_t bytes) {
        void *q = nullptr;
        hipError_t e = hipMalloc(&q, bytes ? bytes : 8);
        if (e != hipSuccess) return fail(QMC_ENOMEM, "hipMalloc (%zu bytes): %s", bytes, hipGetErrorString(e));
        ptr.push_back(q);
        return QMC_OK;
    }
    ~DeviceScratch() {
        for (void *q : ptr) (void)hipFree(q);
    }
};

}  // namespace qmc
