// emd_internal.h -- device-side data structures and helpers of the MI355X EMD
// library (not part of the public ABI).
//
// Solver state layout in HBM.  Every field of the solve (source s, flux components
// u^x and u^t, potential phi, previous residual R) lives in the plan's workspace in
// a padded copy of the batch: gather g occupies [poff, poff + nr * ld) with row
// pitch ld = nt rounded up to a multiple of 32 elements, time contiguous, so that
// every row starts on a 128-byte cache line and each lane's 16-byte vector is
// aligned.  u, phi and R are double-buffered:
// sweep n reads buffer (n & 1) and writes buffer ((n & 1) ^ 1), so neighbouring
// tiles that read halo rows never see a half-updated iterate.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "emd_tiling.h"  // OUT_LANES, GatherMeta, Tile

namespace emd {

// Per-gather status codes (same values as EMD_GATHER_* in the public header).
enum : int {
    ST_RUNNING = 0,
    ST_CONVERGED = 1,
    ST_MAX_ITER = 2,
    ST_ZERO_SOURCE = 3,
    ST_NONFINITE = 4,
    ST_LS_FAIL = 5,
    ST_MASS_IMBALANCE = 6
};

enum : int { LS_L2 = 0, LS_L1 = 1, LS_FIXED = 2, LS_REPLAY = 3 };
enum : int { MASS_BALANCE = 0, MASS_UNIT = 1, MASS_NONE = 2 };

// Number of partial sums a tile contributes to its gather per sweep:
// <A,A>, <A,B>, <B,B>, <grad A,grad A>, <grad A,grad B>, <grad B,grad B>,
// sum |u|, sum u^2 (A = div u_new + s, B = A - previous A).
constexpr int NPART = 8;
// The l1 linesearch test is not a quadratic form in theta, so a sweep sums it for
// NL1 candidate steps at once.  Record layout (NPART_L1 doubles): <A,A>, sum |u|,
// sum u^2, 0, then sum |A + theta_m B| and sum |grad (A + theta_m B)| for the NL1
// candidates theta_m.
constexpr int NL1 = 6;
constexpr int NPART_L1 = 16;
constexpr int WAVE = 64;

// Per-gather scalar state, double-buffered by sweep parity.
struct GState {
    double alpha;      // alpha_k: step of the most recent primal update
    double theta;      // theta_k
    double snorm;      // ||s||_2
    double alpha_max;  // cap on alpha
    double rel_res;    // residual of the flux returned so far
    double emd, transport;  // dx dt Phi(u) and dx dt ||u||_1 of that flux
    int32_t iters;     // accepted iterations
    int32_t status;
    int32_t trials;    // backtracking steps so far
    int32_t started;   // 0 until the first primal update has been applied
    int32_t ubuf;      // buffer holding the returned u once status != RUNNING
    int32_t phibuf;    // buffer holding the returned phi once status != RUNNING
    int32_t flip;      // the gather's fields sit in buffers (sweep parity ^ flip)
    int32_t ls_base;   // l1 linesearch: index of the first candidate in the partials
};

// Where a resumed solve continues a gather from (the checkpointed iteration), or
// the outcome it keeps if the gather had finished.
struct ResumeRec {
    double alpha, theta;
    int32_t iters, trials, status, pad;
    double rel_res, primal, transport;
};

struct SolveScalars {
    double eps, xi, zeta, delta, tol_res;
    int32_t max_iter, check_every, max_ls_trials, ls_mode;
    const double* replay;  // LS_REPLAY: [ngather][ld_replay] accepted steps
    int32_t ld_replay, pad;
    double* hist;          // NULL or [ngather][hist_cap]: residual at every check, a ring
    int32_t hist_cap, pad2;
};

// ---------------------------------------------------------------- reductions

// Data-parallel primitives (DPP): operand modifiers of the vector ALU that read
// another lane of the wavefront, instead of a permute through the LDS.
//   wave_shr:1  (dpp_ctrl 0x138): lane i reads lane i - 1; lane 0 reads 0
//   wave_shl:1  (dpp_ctrl 0x130): lane i reads lane i + 1; lane 63 reads 0
//   row_shr:n   (0x110 + n): lane i reads lane i - n of its row of 16; 0 before it
//   row_bcast:15 / :31 (0x142 / 0x143): rows 1 and 3 read lane 15 of the row before
//     them / rows 2 and 3 read lane 31 (the other rows keep the `old` operand, 0)
template <int CTRL, int ROW_MASK, bool BOUND>
__device__ __forceinline__ int dpp_i(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, 0xF, BOUND);
}

template <int CTRL, int ROW_MASK = 0xF, bool BOUND = true>
__device__ __forceinline__ float dpp(float v)
{
    return __int_as_float(dpp_i<CTRL, ROW_MASK, BOUND>(__float_as_int(v)));
}

template <int CTRL, int ROW_MASK = 0xF, bool BOUND = true>
__device__ __forceinline__ double dpp(double v)
{
    const int lo = dpp_i<CTRL, ROW_MASK, BOUND>(__double2loint(v));
    const int hi = dpp_i<CTRL, ROW_MASK, BOUND>(__double2hiint(v));
    return __hiloint2double(hi, lo);
}

// The value of the previous / next lane (the neighbouring time samples of the
// sweep's lanes); the first / last lane of the wave receives 0.
template <typename T>
__device__ __forceinline__ T lane_prev(T v) { return dpp<0x138>(v); }
template <typename T>
__device__ __forceinline__ T lane_next(T v) { return dpp<0x130>(v); }

// Sum over the 64 lanes of a wavefront, in a fixed order: inclusive prefix sums
// inside each row of 16 lanes (row_shr 1, 2, 4, 8), the row totals carried across
// rows (row_bcast 15, then 31), and lane 63's total moved to scalar registers, so
// every lane (and every wave that reduces the same data) gets the same bits.  All 64
// lanes must be active.
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp<0x111>(v);
    v += dpp<0x112>(v);
    v += dpp<0x114>(v);
    v += dpp<0x118>(v);
    v += dpp<0x142, 0xA, false>(v);
    v += dpp<0x143, 0xC, false>(v);
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

// Sum n records of NP doubles (record p at src[p * NP]) in a fixed order: lane l
// adds records l, l + 64, ... in sequence, then the butterfly.
template <int NP>
__device__ __forceinline__ void reduce_records(const double* __restrict__ src, int n,
                                               double (&out)[NP])
{
    const int lane = threadIdx.x & (WAVE - 1);
    double acc[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) acc[q] = 0.0;
    for (int p = lane; p < n; p += WAVE) {
#pragma unroll
        for (int q = 0; q < NP; ++q) acc[q] += src[(int64_t)p * NP + q];
    }
#pragma unroll
    for (int q = 0; q < NP; ++q) out[q] = wave_sum(acc[q]);
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// A double every lane holds the same value of, moved to scalar registers.
__device__ __forceinline__ double uniform_d(double v)
{
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
    return __hiloint2double(hi, lo);
}

// Blocks are dispatched round-robin over the 8 XCDs (block b on XCD b % 8).  Give
// each XCD a contiguous range of logical blocks (one run of the tile table), so that
// tiles adjacent in the table share that XCD's L2.  gridDim.x is a multiple of 8.
__device__ __forceinline__ int xcd_logical_block()
{
    const int b = blockIdx.x;
    const int per = gridDim.x >> 3;
    return (b & 7) * per + (b >> 3);
}

template <typename T> struct Vec;
template <> struct Vec<float> { using type = float4; static constexpr int N = 4; };
template <> struct Vec<double> { using type = double2; static constexpr int N = 2; };

template <typename T>
__device__ __forceinline__ void vload(const T* __restrict__ p, T (&x)[Vec<T>::N])
{
    using VT = typename Vec<T>::type;
    VT v = *reinterpret_cast<const VT*>(p);
    if constexpr (Vec<T>::N == 4) {
        x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
    } else {
        x[0] = v.x; x[1] = v.y;
    }
}

template <typename T>
__device__ __forceinline__ void vstore(T* __restrict__ p, const T (&x)[Vec<T>::N])
{
    using VT = typename Vec<T>::type;
    VT v;
    if constexpr (Vec<T>::N == 4) {
        v.x = x[0]; v.y = x[1]; v.z = x[2]; v.w = x[3];
    } else {
        v.x = x[0]; v.y = x[1];
    }
    *reinterpret_cast<VT*>(p) = v;
}

}  // namespace emd
