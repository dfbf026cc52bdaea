// Level kernel of synchronous parallel simulated annealing for gfx950.
//
// One Markov chain per lane.  A workgroup of WG lanes keeps a tile of chains'
// states in LDS as x[d][lane] (coordinate-major), so a per-lane random
// coordinate d is a bank-conflict-free LDS access.  One launch runs one
// temperature level (Sec. 2.2.2: every chain runs N Metropolis steps at a
// fixed T and the lowest final state starts every chain at the next level).
// Each workgroup runs its tiles of chains, keeps its best chain, re-evaluates
// that state in full and publishes it as a candidate with plain stores; the
// kernel boundary makes the candidates visible, and every workgroup of the
// next level's launch reduces them to the same winner before it starts.
// There is no cross-workgroup synchronisation inside a launch: on gfx950 a
// grid-wide barrier (or a last-workgroup hand-off with agent-scope fences)
// costs several times the ~1.5 us of a graph-replayed launch.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>

#include "sa_device.hpp"
#include "sa_internal.hpp"
#include "sa_step.hpp"
#include "sa_level_common.hpp"
#include "sa_level_kernel.hpp"

namespace sa {

// Close a run of levels: reduce the last level's candidates and publish its
// trace entry, record and broadcast state.
template <typename R>
__global__ void __launch_bounds__(256) finalize_kernel(const LevelArgs<R> a, const uint32_t level,
                                                        const uint32_t groups)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ Slot<R> wave_slot[4];
    __shared__ uint64_t wave_acc[4];
    __shared__ double sh_start[3];
    adopt_winner<R>(a, level, groups, reinterpret_cast<R *>(lds_raw), sh_start, true, wave_slot, wave_acc);
}

__global__ void reset_kernel(double *rec, uint32_t *rec_level, double *elite_f)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        rec[0] = __builtin_inf();
        *rec_level = 0xFFFFFFFFu;
        elite_f[0] = __builtin_inf();
        elite_f[3] = __builtin_inf();
    }
}

size_t level_lds_bytes(uint32_t n, uint32_t wg, size_t real_size, bool table, bool learn)
{
    return ((size_t)n * wg + 2 * (size_t)n + (table ? 4 * (size_t)n : 0)) * real_size +
           (learn ? (size_t)mlp::kNetBytes : 0);
}

template <typename R, int F, bool TABLE, int MODE, int MOVE, bool UNSHIFTED = false>
static hipError_t launch_one(const LevelArgs<R> &a, uint32_t level, uint32_t prev_groups, uint32_t *groups,
                             hipStream_t s)
{
    auto kern = level_kernel<R, F, TABLE, MODE, MOVE, UNSHIFTED>;
    const size_t lds =
        level_lds_bytes(a.n, a.wg, sizeof(R), TABLE, MODE >= kModeLearn);
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, (int)a.wg, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    const uint32_t grid = (uint32_t)std::min<uint64_t>((uint64_t)per_cu * a.num_cus, a.tiles);
    *groups = grid;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(a.wg), lds, s, a, level, prev_groups);
    return hipGetLastError();
}

template <typename R, int F, bool TABLE, int MOVE>
static hipError_t launch_mode(int mode, const LevelArgs<R> &a, uint32_t level, uint32_t prev, uint32_t *groups,
                              hipStream_t s)
{
    switch (mode) {
    case kModePlain:
        if constexpr (!TABLE && sizeof(R) == sizeof(float)) {
            if (a.sh == R(0) && !std::signbit(a.sh) && a.exchange == 1)  // +0 exactly, synchronous
                return launch_one<R, F, TABLE, kModePlain, MOVE, true>(a, level, prev, groups, s);
        }
        return launch_one<R, F, TABLE, kModePlain, MOVE>(a, level, prev, groups, s);
    case kModeLog: return launch_one<R, F, TABLE, kModeLog, MOVE>(a, level, prev, groups, s);
    case kModeCapture: return launch_one<R, F, TABLE, kModeCapture, MOVE>(a, level, prev, groups, s);
    default: break;
    }
    if constexpr (sizeof(R) == sizeof(float) && MOVE == SA_MOVE_RADIUS) {
        if (mode == kModeLearn) return launch_one<R, F, TABLE, kModeLearn, MOVE>(a, level, prev, groups, s);
        if (mode == kModeLearnLog) return launch_one<R, F, TABLE, kModeLearnLog, MOVE>(a, level, prev, groups, s);
        if (mode == kModeLearnG) return launch_one<R, F, TABLE, kModeLearnG, MOVE>(a, level, prev, groups, s);
        if (mode == kModeLearnLogG) return launch_one<R, F, TABLE, kModeLearnLogG, MOVE>(a, level, prev, groups, s);
    }
    return hipErrorInvalidValue;
}

template <typename R, int F>
static hipError_t dispatch_f(bool table, int mode, const LevelArgs<R> &a, uint32_t level, uint32_t prev,
                             uint32_t *groups, hipStream_t s)
{
    if (a.move == SA_MOVE_RADIUS)
        return table ? launch_mode<R, F, true, SA_MOVE_RADIUS>(mode, a, level, prev, groups, s)
                     : launch_mode<R, F, false, SA_MOVE_RADIUS>(mode, a, level, prev, groups, s);
    return table ? launch_mode<R, F, true, SA_MOVE_RESAMPLE>(mode, a, level, prev, groups, s)
                 : launch_mode<R, F, false, SA_MOVE_RESAMPLE>(mode, a, level, prev, groups, s);
}

template <typename R>
static hipError_t dispatch(int func, bool table, int mode, const LevelArgs<R> &a, uint32_t level, uint32_t prev,
                           uint32_t *groups, hipStream_t s)
{
    switch (func) {
    case kSchwefel: return dispatch_f<R, kSchwefel>(table, mode, a, level, prev, groups, s);
    case kRastrigin: return dispatch_f<R, kRastrigin>(table, mode, a, level, prev, groups, s);
    case kAckley: return dispatch_f<R, kAckley>(table, mode, a, level, prev, groups, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_level_f32(int func, bool table, int mode, const LevelArgs<float> &a, uint32_t level,
                            uint32_t prev_groups, uint32_t *groups, hipStream_t s)
{
    return dispatch<float>(func, table, mode, a, level, prev_groups, groups, s);
}

hipError_t launch_level_f64(int func, bool table, int mode, const LevelArgs<double> &a, uint32_t level,
                            uint32_t prev_groups, uint32_t *groups, hipStream_t s)
{
    return dispatch<double>(func, table, mode, a, level, prev_groups, groups, s);
}

hipError_t launch_finalize_f32(const LevelArgs<float> &a, uint32_t level, uint32_t groups, hipStream_t s)
{
    hipLaunchKernelGGL(finalize_kernel<float>, dim3(1), dim3(256), a.n * sizeof(float), s, a, level, groups);
    return hipGetLastError();
}

hipError_t launch_finalize_f64(const LevelArgs<double> &a, uint32_t level, uint32_t groups, hipStream_t s)
{
    hipLaunchKernelGGL(finalize_kernel<double>, dim3(1), dim3(256), a.n * sizeof(double), s, a, level, groups);
    return hipGetLastError();
}

hipError_t launch_reset(double *rec, uint32_t *rec_level, double *elite_f, hipStream_t s)
{
    hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(64), 0, s, rec, rec_level, elite_f);
    return hipGetLastError();
}

}  // namespace sa
