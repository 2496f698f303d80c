// Registry of compiled lattice-kernel instantiations.
//
// Each (family, transform, dimension, shift tile) combination is a separate
// template instantiation, compiled in its own translation unit; those units
// register a launcher here when the library is loaded.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <tuple>

#include "qmc_kernels.hpp"

namespace qmc {

// internal family codes: the public qmc_family values, plus the complex
// sector integrand as its own code
enum : int { kFamSectorComplex = 100 };

struct KernelKey {
    int family;  // qmc_family value or kFamSectorComplex
    int tkind;   // 0 none, 1 Korobov, 2 baker
    int alpha;   // Korobov weight (0 otherwise)
    int d;
    int T;
    bool operator<(const KernelKey &o) const {
        return std::tie(family, tkind, alpha, d, T) < std::tie(o.family, o.tkind, o.alpha, o.d, o.T);
    }
};

using LatticeLaunch = hipError_t (*)(const LatticeArgs &, dim3 grid, hipStream_t);

std::map<KernelKey, LatticeLaunch> &lattice_registry();

struct LatticeRegistrar {
    LatticeRegistrar(KernelKey k, LatticeLaunch f) { lattice_registry()[k] = f; }
};

template <class Fam, class Tr, int D, int T>
hipError_t launch_lattice(const LatticeArgs &a, dim3 grid, hipStream_t s) {
    hipLaunchKernelGGL((k_lattice<Fam, Tr, D, T>), grid, dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

struct BatchKey {
    int family, tkind, alpha, d, T;
    bool operator<(const BatchKey &o) const {
        return std::tie(family, tkind, alpha, d, T) < std::tie(o.family, o.tkind, o.alpha, o.d, o.T);
    }
};

// persistent = 1: `blocks` workgroups loop over the work list; 0: one
// workgroup per tile (blocks ignored)
using BatchLaunch = hipError_t (*)(const BatchArgs &, uint32_t blocks, int persistent, hipStream_t);

std::map<BatchKey, BatchLaunch> &batch_registry();

struct BatchRegistrar {
    BatchRegistrar(BatchKey k, BatchLaunch f) { batch_registry()[k] = f; }
};

template <class Fam, class Tr, int D, int T>
hipError_t launch_batch(const BatchArgs &a, uint32_t blocks, int persistent, hipStream_t s) {
    if (persistent)
        hipLaunchKernelGGL((k_batch<Fam, Tr, D, T>), dim3(blocks), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL((k_batch_flat<Fam, Tr, D, T>), dim3(a.ntiles), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

// launchers of the non-templated helper kernels (qmc_common.hip)
hipError_t launch_finalize(const FinalizeArgs &a, uint32_t ninst, hipStream_t s);
hipError_t launch_dump(const DumpArgs &a, uint32_t blocks, hipStream_t s);
hipError_t launch_math(int fn, uint64_t count, const double *x, double *y, hipStream_t s);
hipError_t launch_zero_u32(uint32_t *p, uint32_t count, hipStream_t s);
hipError_t launch_finalize_batch(const FinalizeBatchArgs &a, uint32_t count, hipStream_t s);

}  // namespace qmc
