// Launchers of the level kernel's exchange variants (Sec. 2.2): the
// stochastic exchange (a reading of the stochastic crossover the paper names
// beside the minimum operator) and the best-seen reduction, on the dense state
// layout with plain or logged moves.  The kernel itself is the level kernel
// of sa_level_kernel.hpp instantiated with VAR != 0; the plain launchers
// (sa_kernels.hip) instantiate VAR = 0, so the variants add no code to them.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "sa_internal.hpp"
#include "sa_level_kernel.hpp"

namespace sa {

size_t variant_lds_bytes(uint32_t n, uint32_t wg, size_t real_size, bool table, bool best_seen, uint32_t steps)
{
    const size_t extra = best_seen ? ((size_t)((steps + 31u) / 32u) * wg + 2 * (size_t)steps) * sizeof(uint32_t) : 0;
    return level_lds_bytes(n, wg, real_size, table, false) + extra;
}

namespace {

template <typename R, int F, bool TABLE, int MODE, int MOVE, int VAR>
hipError_t launch_one(const LevelArgs<R> &a, uint32_t level, uint32_t prev_groups, uint32_t *groups, hipStream_t s)
{
    auto kern = level_kernel<R, F, TABLE, MODE, MOVE, false, VAR>;
    const size_t lds = variant_lds_bytes(a.n, a.wg, sizeof(R), TABLE, (VAR & kVarBest) != 0, a.steps);
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, (int)a.wg, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    const uint32_t grid = (uint32_t)std::min<uint64_t>((uint64_t)per_cu * a.num_cus, a.tiles);
    *groups = grid;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(a.wg), lds, s, a, level, prev_groups);
    return hipGetLastError();
}

template <typename R, int F, bool TABLE, int MOVE, int VAR>
hipError_t launch_log(bool log, const LevelArgs<R> &a, uint32_t level, uint32_t prev, uint32_t *groups,
                      hipStream_t s)
{
    return log ? launch_one<R, F, TABLE, kModeLog, MOVE, VAR>(a, level, prev, groups, s)
               : launch_one<R, F, TABLE, kModePlain, MOVE, VAR>(a, level, prev, groups, s);
}

template <typename R, int F, bool TABLE, int MOVE>
hipError_t launch_var(int var, bool log, const LevelArgs<R> &a, uint32_t level, uint32_t prev, uint32_t *groups,
                      hipStream_t s)
{
    switch (var) {
    case kVarSos: return launch_log<R, F, TABLE, MOVE, kVarSos>(log, a, level, prev, groups, s);
    case kVarBest: return launch_log<R, F, TABLE, MOVE, kVarBest>(log, a, level, prev, groups, s);
    case kVarSos | kVarBest: return launch_log<R, F, TABLE, MOVE, kVarSos | kVarBest>(log, a, level, prev, groups, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename R, int F>
hipError_t dispatch_f(bool table, int var, bool log, const LevelArgs<R> &a, uint32_t level, uint32_t prev,
                      uint32_t *groups, hipStream_t s)
{
    if (a.move == SA_MOVE_RADIUS)
        return table ? launch_var<R, F, true, SA_MOVE_RADIUS>(var, log, a, level, prev, groups, s)
                     : launch_var<R, F, false, SA_MOVE_RADIUS>(var, log, a, level, prev, groups, s);
    return table ? launch_var<R, F, true, SA_MOVE_RESAMPLE>(var, log, a, level, prev, groups, s)
                 : launch_var<R, F, false, SA_MOVE_RESAMPLE>(var, log, a, level, prev, groups, s);
}

template <typename R>
hipError_t dispatch(int func, bool table, int var, bool log, const LevelArgs<R> &a, uint32_t level, uint32_t prev,
                    uint32_t *groups, hipStream_t s)
{
    switch (func) {
    case kSchwefel: return dispatch_f<R, kSchwefel>(table, var, log, a, level, prev, groups, s);
    case kRastrigin: return dispatch_f<R, kRastrigin>(table, var, log, a, level, prev, groups, s);
    case kAckley: return dispatch_f<R, kAckley>(table, var, log, a, level, prev, groups, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_variant_level_f32(int func, bool table, int var, bool log, const LevelArgs<float> &a,
                                    uint32_t level, uint32_t prev_groups, uint32_t *groups, hipStream_t s)
{
    return dispatch<float>(func, table, var, log, a, level, prev_groups, groups, s);
}

hipError_t launch_variant_level_f64(int func, bool table, int var, bool log, const LevelArgs<double> &a,
                                    uint32_t level, uint32_t prev_groups, uint32_t *groups, hipStream_t s)
{
    return dispatch<double>(func, table, var, log, a, level, prev_groups, groups, s);
}

}  // namespace sa
