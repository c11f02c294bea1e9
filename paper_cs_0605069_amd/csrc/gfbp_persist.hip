// Persistent work-list kernels (one per field, degree class and schedule) and
// their launcher; compiled apart from gfbp.hip so the two build in parallel.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/gfbp.h"
#include "gfbp_kernels.h"
#include "gfbp_tiled.h"
#include "gfbp_persist.h"

namespace gfbp {
namespace persist {

namespace {

template <int P, int LEL, int DCM, int DVM, int SCH>
hipError_t launch_one(const Group *groups, const Work *work, int n_work, uint32_t *next, const Batch &B, int waves,
                      hipStream_t st, hipEvent_t a, hipEvent_t b) {
    auto kern = k_persist<P, LEL, DCM, DVM, SCH>;
    constexpr int LG = Pick<P, LEL>::LG;
    const int block = waves * kWave;
    const size_t lds = size_t(waves) * tiled::Geo<P, LG>::PERM * sizeof(float);
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, block, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    const unsigned grid = unsigned(std::min<long long>(n_work, (long long)cus * per_cu));
    if (a) hipExtLaunchKernelGGL(kern, dim3(grid), dim3(block), uint32_t(lds), st, a, b, 0, groups, work, n_work, next, B);
    else hipLaunchKernelGGL(kern, dim3(grid), dim3(block), uint32_t(lds), st, groups, work, n_work, next, B);
    return hipGetLastError();
}

template <int P, int SCH>
hipError_t launch_p(int lel, bool small, const Group *groups, const Work *work, int n_work, uint32_t *next,
                    const Batch &B, int waves, hipStream_t st, hipEvent_t a, hipEvent_t b) {
    if constexpr (P == 2 || P == 3) {  // two entries per lane: the small fields' 16- and 32-frame tiles
        if (lel == 1 && !small) return launch_one<P, 1, 16, 8, SCH>(groups, work, n_work, next, B, waves, st, a, b);
        if (lel == 1) return launch_one<P, 1, 6, 4, SCH>(groups, work, n_work, next, B, waves, st, a, b);
    }
    if (!small) return launch_one<P, 2, 16, 8, SCH>(groups, work, n_work, next, B, waves, st, a, b);
    if (lel == 3) return launch_one<P, 3, 6, 4, SCH>(groups, work, n_work, next, B, waves, st, a, b);
    return launch_one<P, 2, 6, 4, SCH>(groups, work, n_work, next, B, waves, st, a, b);
}

template <int SCH>
hipError_t launch_s(int p, int lel, bool small, const Group *groups, const Work *work, int n_work, uint32_t *next,
                    const Batch &B, int waves, hipStream_t st, hipEvent_t a, hipEvent_t b) {
    switch (p) {
        case 1: return launch_p<1, SCH>(lel, small, groups, work, n_work, next, B, waves, st, a, b);
        case 2: return launch_p<2, SCH>(lel, small, groups, work, n_work, next, B, waves, st, a, b);
        case 3: return launch_p<3, SCH>(lel, small, groups, work, n_work, next, B, waves, st, a, b);
        case 4: return launch_p<4, SCH>(lel, small, groups, work, n_work, next, B, waves, st, a, b);
        case 5: return launch_p<5, SCH>(lel, small, groups, work, n_work, next, B, waves, st, a, b);
        case 6: return launch_p<6, SCH>(lel, small, groups, work, n_work, next, B, waves, st, a, b);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_persistent(int p, int lel, bool small, int sch, const Group *groups, const Work *work, int n_work,
                             uint32_t *next, const Batch &B, int waves, hipStream_t st, hipEvent_t a, hipEvent_t b) {
    if (n_work <= 0) return hipSuccess;
    if (waves < 1 || waves > 8 || lel < 1 || lel > 3) return hipErrorInvalidValue;
    if (sch == GFBP_PUS) return launch_s<GFBP_PUS>(p, lel, small, groups, work, n_work, next, B, waves, st, a, b);
    return launch_s<GFBP_SUS>(p, lel, small, groups, work, n_work, next, B, waves, st, a, b);
}

}  // namespace persist
}  // namespace gfbp
