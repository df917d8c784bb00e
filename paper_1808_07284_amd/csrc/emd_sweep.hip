// emd_sweep.hip -- the fused PDHG-with-linesearch sweep (Algorithm 1 of the paper,
// Section 2.2), one launch per iteration for every gather of the batch.
//
// Iteration k of the paper is
//   u_{k+1}   = shrink(u_k + alpha_k grad phi_k, alpha_k) / (1 + eps alpha_k)
//   choose alpha_{k+1} (linesearch), theta_{k+1} = alpha_{k+1}/alpha_k,
//   beta_{k+1} = delta alpha_{k+1}
//   phi_{k+1} = phi_k + beta_{k+1} (div ubar + s),  ubar = u_{k+1} + theta (u_{k+1} - u_k).
// With A_m = div u_m + s the dual step is phi_k + beta (A_{k+1} + theta B_{k+1}),
// B_{k+1} = A_{k+1} - A_k, so the linesearch test of Algorithm 1 in Euclidean norms,
//   delta alpha^2 ||grad(A + theta B)||^2 <= zeta^2 ||A + theta B||^2,
// is a scalar inequality in the six inner products <A,A>, <A,B>, <B,B>,
// <gA,gA>, <gA,gB>, <gB,gB>: every backtracking trial is free once they are known.
//
// Sweep n therefore (1) reduces the previous sweep's per-tile partials of those
// products and decides alpha_n, theta_n, beta_n and the stop rule (every wave of a
// gather does this redundantly, in a fixed order, so all agree bitwise; the four
// waves of a block on one gather share the summing),
// (2) applies the dual step of iteration n-1 -> n, (3) the primal update with
// alpha_n, (4) recomputes div of the new flux and the six products plus
// sum |u|, sum u^2 for the next decision.  One HBM pass per iteration: read u, phi,
// s, R (the previous residual A_n), write u, phi, R -- 36 bytes per cell in FP32.
//
// Work decomposition: a wavefront owns a tile of `rows` receiver rows by 56 * V
// time samples (V = 4 floats or 2 doubles per lane, one 16-byte vector per field).
// Lanes run along time (coalesced), the wave marches along the rows keeping the
// neighbouring rows in registers: down on even strips, up on odd ones, so that two
// tiles sharing halo rows read them at about the same time (see PipeUp).  The
// operators couple a cell to its neighbours at distance <= 2 rows above and 1 row
// below, and 2 samples back / 1 ahead in time: rows are recomputed for the halo
// (2 rows above the tile and 1 below), and lanes 0 and 57 carry the time halo
// (their own samples are loaded and computed but never stored or reduced); lanes
// 58..63 neither load nor store.
#include <type_traits>

#include "emd_internal.h"
#include "emd_launch.h"

namespace emd {

struct Decision {
    double alpha;  // primal step of this sweep
    double beta;   // dual step of this sweep (0: no dual update)
    double theta;
    int run;       // 0: gather finished, nothing to do
    int prox;      // 1: compute the next primal iterate and its reductions
    int eval;      // 1 (l1 test only): no candidate passed; re-evaluate the next ones
    double cand0;  // l1 test: first candidate step of the next decision ...
    double cand_ref;  // ... and the step its theta is relative to
};

// First candidate step of a linesearch from step ak and theta tk, after `skip`
// backtracking factors; the sweep and the decision compute the candidates with
// the same operations, so they agree bitwise.
__device__ __forceinline__ double first_candidate(double ak, double tk, double amax, double xi, int skip)
{
    double alpha = ak * sqrt(1.0 + tk);
    if (alpha > amax) alpha = amax;
    for (int m = 0; m < skip; ++m) alpha *= xi;
    return alpha;
}

// The fixed order in which a gather's decision sums its tiles' records, so that
// every wave forming it, under any tiling and any narrowing of the table, gets the
// same bits: record p goes to quarter (p / 64) % 4 and lane p % 64; each lane adds
// its records of a quarter in slot order, the quarter's lanes are added by
// wave_sum, and the quarters are added in order ((S0 + S1) + S2) + S3.
template <int NP>
__device__ __forceinline__ void quarter_sum(const double* __restrict__ src, int n, int w,
                                            double (&s)[NP])
{
    const int lane = threadIdx.x & (WAVE - 1);
    double acc[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) acc[q] = 0.0;
    for (int p = w * WAVE + lane; p < n; p += 4 * WAVE) {
#pragma unroll
        for (int q = 0; q < NP; ++q) acc[q] += src[(int64_t)p * NP + q];
    }
#pragma unroll
    for (int q = 0; q < NP; ++q) s[q] = wave_sum(acc[q]);
}

// red != NULL: the four waves of this block each sum one quarter (wave w, quarter w)
// and exchange them through red (LDS, 4 * NP doubles) at one block barrier that
// every wave of the block reaches; otherwise this wave sums all four quarters.
template <int NP>
__device__ __forceinline__ void decision_sums(const double* __restrict__ src, int n, int w,
                                              double* red, double (&out)[NP])
{
    if (red) {
        double s[NP];
        quarter_sum<NP>(src, n, w, s);
        if ((threadIdx.x & (WAVE - 1)) == 0) {
#pragma unroll
            for (int q = 0; q < NP; ++q) red[w * NP + q] = s[q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NP; ++q) out[q] = ((red[q] + red[NP + q]) + red[2 * NP + q]) + red[3 * NP + q];
    } else {
        double s[NP];
        quarter_sum<NP>(src, n, 0, out);
        for (int k = 1; k < 4; ++k) {
            quarter_sum<NP>(src, n, k, s);
#pragma unroll
            for (int q = 0; q < NP; ++q) out[q] += s[q];
        }
    }
}

// Runs on every lane of a wave; returns the same decision on every lane.
// ABS: the l1 form of the linesearch test (records of NPART_L1 doubles).
// pb: buffer parity of the gather's fields in this sweep.  w, red: this wave's index
// in its block and the block's exchange buffer for the record sums (see
// decision_sums; NULL when the wave sums alone).
template <typename T, bool ABS>
__device__ Decision decide(const SweepArgs<T>& a, int p, int g, const GatherMeta& gm,
                           bool writer, int pb, int w, double* red)
{
    const GState* __restrict__ sin = a.gst[p] + g;
    GState* __restrict__ sout = a.gst[p ^ 1] + g;
    GState st = *sin;
    const SolveScalars& sc = a.sc;
    Decision d;
    d.alpha = st.alpha;
    d.beta = 0.0;
    d.theta = 0.0;
    d.run = 0;
    d.prox = 0;
    d.eval = 0;
    d.cand0 = 0.0;
    d.cand_ref = 1.0;
    const int lane = threadIdx.x & (WAVE - 1);
    if (st.status != ST_RUNNING) {
        if (writer && lane == 0) *sout = st;
        return d;
    }
    if (!st.started) {
        // iteration 1: primal update from (u_1, phi_1) with alpha_1, no dual step yet
        st.started = 1;
        if (writer && lane == 0) *sout = st;
        d.run = 1;
        d.prox = 1;
        if constexpr (ABS) {
            d.cand0 = first_candidate(st.alpha, st.theta, st.alpha_max, sc.xi, 0);
            d.cand_ref = st.alpha;
        }
        return d;
    }
    constexpr int NP = ABS ? NPART_L1 : NPART;
    double q[NP];
    decision_sums<NP>(a.part[p] + (int64_t)gm.tile_base * NP, gm.ntiles, w, red, q);
    const double aa = q[0];
    const double l1 = ABS ? q[1] : q[6], l2 = ABS ? q[2] : q[7];
    const double ak = st.alpha, tk = st.theta;
    double alpha, theta = 1.0;
    int trials = 0, status = ST_RUNNING;
    bool finite = true;
#pragma unroll
    for (int m = 0; m < NP; ++m) finite = finite && isfinite(q[m]);
    if (!finite) {
        status = ST_NONFINITE;
        alpha = ak;
    } else if constexpr (ABS) {
        // candidates ls_base, ls_base + 1, ... of this iteration's backtracking:
        //   sqrt(delta) alpha ||grad rbar||_1 <= zeta ||rbar||_1,  rbar = A + theta B
        alpha = first_candidate(ak, tk, st.alpha_max, sc.xi, st.ls_base);
        const double sd = sqrt(sc.delta);
        bool found = false;
        for (int m = 0; m < NL1 && status == ST_RUNNING; ++m) {
            theta = alpha / ak;
            const double lhs = sd * alpha * q[4 + NL1 + m];
            const double rhs = sc.zeta * q[4 + m];
            if (!(isfinite(lhs) && isfinite(rhs))) {
                status = ST_NONFINITE;
                break;
            }
            if (lhs <= rhs) {
                found = true;
                break;
            }
            alpha *= sc.xi;
            ++trials;
            if (st.ls_base + trials > sc.max_ls_trials) status = ST_LS_FAIL;
        }
        if (!found && status == ST_RUNNING) {
            // every candidate of the record failed: an evaluation sweep sums the
            // next NL1 for the same flux; the fields stay where they are, so the
            // following sweep reads the other buffer parity
            st.trials += trials;
            st.ls_base += NL1;
            st.flip ^= 1;
            if (writer && lane == 0) *sout = st;
            d.run = 1;
            d.eval = 1;
            d.cand0 = first_candidate(ak, tk, st.alpha_max, sc.xi, st.ls_base);
            d.cand_ref = ak;
            return d;
        }
    } else if (sc.ls_mode == LS_FIXED) {
        alpha = ak;
        theta = 1.0;
    } else if (sc.ls_mode == LS_REPLAY) {
        alpha = sc.replay[(int64_t)g * sc.ld_replay + st.iters];
        theta = alpha / ak;
    } else {
        const double ab = q[1], bb = q[2], gaa = q[3], gab = q[4], gbb = q[5];
        alpha = ak * sqrt(1.0 + tk);
        if (alpha > st.alpha_max) alpha = st.alpha_max;
        for (;;) {
            theta = alpha / ak;
            const double lhs = sc.delta * alpha * alpha * (gaa + 2.0 * theta * gab + theta * theta * gbb);
            const double rhs = sc.zeta * sc.zeta * (aa + 2.0 * theta * ab + theta * theta * bb);
            if (!(isfinite(lhs) && isfinite(rhs))) {
                status = ST_NONFINITE;
                break;
            }
            if (lhs <= rhs) break;
            alpha *= sc.xi;
            ++trials;
            if (trials > sc.max_ls_trials) {
                status = ST_LS_FAIL;
                break;
            }
        }
    }
    st.trials += trials;
    st.ls_base = 0;
    const int qb = pb ^ 1;
    if (status == ST_RUNNING) {
        // accept iteration st.iters + 1: phi_n is written by this sweep, u_n is the
        // flux this sweep reads
        st.iters += 1;
        st.rel_res = sqrt(aa) / st.snorm;
        st.emd = gm.cm * (l1 + 0.5 * sc.eps * l2);
        st.transport = gm.cm * l1;
        st.alpha = alpha;
        st.theta = theta;
        if (sc.hist && writer && lane == 0 && st.iters % sc.check_every == 0)
            sc.hist[(int64_t)g * sc.hist_cap + (st.iters / sc.check_every - 1) % sc.hist_cap] = st.rel_res;
        if (st.iters % sc.check_every == 0 && st.rel_res <= sc.tol_res) status = ST_CONVERGED;
        else if (st.iters >= sc.max_iter) status = ST_MAX_ITER;
        d.run = 1;
        d.prox = (status == ST_RUNNING);
        d.alpha = alpha;
        d.beta = sc.delta * alpha;
        d.theta = theta;
        st.ubuf = pb;
        st.phibuf = qb;
        if constexpr (ABS) {
            d.cand0 = first_candidate(alpha, theta, st.alpha_max, sc.xi, 0);
            d.cand_ref = alpha;
        }
    } else {
        // the trial step is rejected: return the last accepted iterate (u_{n-1} is
        // still in the buffer this sweep would have written, phi_{n-1} in its input)
        st.ubuf = qb;
        st.phibuf = pb;
    }
    st.status = status;
    if (writer && lane == 0) {
        *sout = st;
        if (status != ST_RUNNING) atomicAdd(a.done, 1);
    }
    return d;
}

template <typename T>
__device__ __forceinline__ T shrink_scaled(T v, T a, T inv)
{
    // shrink(v, a) = (1 - a/|v|) v for |v| >= a, else 0 (Section 2.2), times
    // 1/(1 + eps a); written as v - a sign(v)
    const T m = fabs(v) - a;
    return m >= T(0) ? copysign(m, v) * inv : T(0);
}

template <typename T>
__device__ __forceinline__ void zero(T (&x)[Vec<T>::N])
{
#pragma unroll
    for (int k = 0; k < Vec<T>::N; ++k) x[k] = T(0);
}

template <typename T>
__device__ __forceinline__ void swap2(bool s, T& x, T& y)
{
    const T a = s ? y : x, b = s ? x : y;
    x = a;
    y = b;
}

// Per-tile constants.  Field accesses go through raw buffer instructions on a
// descriptor spanning the gather's padded region of that field: a lane or row that
// must not touch memory gets an offset beyond the region, for which the hardware
// returns zeros (loads) or drops the access (stores).  So every load and store is
// issued unconditionally and the compiler can count them exactly in s_waitcnt.
template <typename T>
struct TileCtx {
    static constexpr int V = Vec<T>::N;
    int nr, ld, r0, rend, ibeg, ilast;
    bool lane_out;
    bool inb[V], jgt0[V], jlt[V];
    T idx, idt, beta, theta, alpha, inv;
    double thm[NL1];               // l1 linesearch: candidate thetas of the next decision
    uint32_t row_bytes;            // ld * sizeof(T)
    uint32_t vb_ld, vb_st;         // lane byte offsets for loads / stores (or OOB)
    __amdgpu_buffer_rsrc_t uxi, uti, phi_i, ri, si, uxo, uto, phio, ro;
};

// Byte offset that is out of range of every gather region (regions are at most
// 1 GiB, row offsets at most 1 GiB + 3 rows), without 32-bit wrap-around.
constexpr uint32_t OOB = 0x40000000u;

template <typename T>
__device__ __forceinline__ void bload(__amdgpu_buffer_rsrc_t r, uint32_t off, T (&x)[Vec<T>::N])
{
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    if constexpr (Vec<T>::N == 4) {
        x[0] = __uint_as_float(v[0]);
        x[1] = __uint_as_float(v[1]);
        x[2] = __uint_as_float(v[2]);
        x[3] = __uint_as_float(v[3]);
    } else {
        x[0] = __hiloint2double((int)v[1], (int)v[0]);
        x[1] = __hiloint2double((int)v[3], (int)v[2]);
    }
}

// Cache policy of the field stores: non-temporal.  A sweep's output is read again
// only by the next sweep, after the whole batch (gigabytes) has streamed through the
// caches, so keeping it there only evicts lines that are still useful: the halo rows
// the neighbouring tiles read shortly after (on the 64-gather batch a steady sweep
// takes ~5 % less time and misses the L2 ~6 % less).  Loads keep the default policy.
constexpr int kStoreNonTemporal = 2;

template <typename T>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t off, const T (&x)[Vec<T>::N])
{
    using U4 = decltype(__builtin_amdgcn_raw_buffer_load_b128(r, 0u, 0, 0));
    U4 v;
    if constexpr (Vec<T>::N == 4) {
        v[0] = __float_as_uint(x[0]);
        v[1] = __float_as_uint(x[1]);
        v[2] = __float_as_uint(x[2]);
        v[3] = __float_as_uint(x[3]);
    } else {
        v[0] = (uint32_t)__double2loint(x[0]);
        v[1] = (uint32_t)__double2hiint(x[0]);
        v[2] = (uint32_t)__double2loint(x[1]);
        v[3] = (uint32_t)__double2hiint(x[1]);
    }
    __builtin_amdgcn_raw_buffer_store_b128(v, r, off, 0, kStoreNonTemporal);
}

// Divergence of a flux on one row plus a source term:
//   ([has_next] wxf - [has_prev] wx) / dx + ([j + 1 < nt] wt_{j+1} - [j > 0] wt_j) / dt + add,
// the forward difference of the paper in the interior and minus the transpose of
// the backward-difference gradient on the last row/column.
template <typename T, bool EDGE>
__device__ __forceinline__ void div_row(const TileCtx<T>& c, bool has_next, bool has_prev,
                                        const T (&wx)[Vec<T>::N], const T (&wxf)[Vec<T>::N],
                                        const T (&wt)[Vec<T>::N], T wt_next,
                                        const T (&add)[Vec<T>::N], T (&out)[Vec<T>::N])
{
    constexpr int V = Vec<T>::N;
    // the row conditions are uniform: fold them into the difference weights
    const T wf = has_next ? c.idx : T(0), wb = has_prev ? c.idx : T(0);
#pragma unroll
    for (int k = 0; k < V; ++k) {
        T ft = (k + 1 < V) ? wt[(k + 1) % V] : wt_next;
        T bt = wt[k];
        if constexpr (EDGE) {
            ft = c.jlt[k] ? ft : T(0);
            bt = c.jgt0[k] ? bt : T(0);
        }
        out[k] = fma(ft - bt, c.idt, fma(wxf[k], wf, fma(-wx[k], wb, add[k])));
    }
}

// Partial sums of one residual cell of the new flux, a = A_{n+1} and b = B_{n+1}:
// the cell's own terms and its time-gradient terms (gat, gbt) ...
template <bool ABS, int NP>
__device__ __forceinline__ void acc_cell(double (&acc)[NP], const double (&thm)[NL1], double av,
                                         double bv, double gat, double gbt)
{
    acc[0] = fma(av, av, acc[0]);
    if constexpr (ABS) {
#pragma unroll
        for (int m = 0; m < NL1; ++m) {
            acc[4 + m] += fabs(fma(thm[m], bv, av));
            acc[4 + NL1 + m] += fabs(fma(thm[m], gbt, gat));
        }
    } else {
        acc[1] = fma(av, bv, acc[1]);
        acc[2] = fma(bv, bv, acc[2]);
        acc[3] = fma(gat, gat, acc[3]);
        acc[4] = fma(gat, gbt, acc[4]);
        acc[5] = fma(gbt, gbt, acc[5]);
    }
}

// ... and its x-gradient terms (gax, gbx)
template <bool ABS, int NP>
__device__ __forceinline__ void acc_xgrad(double (&acc)[NP], const double (&thm)[NL1], double gax,
                                          double gbx)
{
    if constexpr (ABS) {
#pragma unroll
        for (int m = 0; m < NL1; ++m) acc[4 + NL1 + m] += fabs(fma(thm[m], gbx, gax));
    } else {
        acc[3] = fma(gax, gax, acc[3]);
        acc[4] = fma(gax, gbx, acc[4]);
        acc[5] = fma(gbx, gbx, acc[5]);
    }
}

// The row pipeline of one wavefront.  Every per-row quantity lives in register
// sets indexed by the row's position relative to the first row (mod 4 for u^x,
// mod 2 for everything else), and the loop is unrolled by four, so no register is
// ever copied and each load writes registers whose previous row is already dead:
//   u^x of row i + 3 is issued at the top of step i (two steps of latency hidden),
//   u^t, phi, s, R of row i + 1 at the top of step i.
// With B_{n+1} = div(u_{n+1} - u_n) and A_{n+1} = A_n + B_{n+1} the residual of the
// new flux on row i - 1 needs only the flux change of rows i - 1 and i and A_n of
// row i - 1 (B is formed from the small flux change instead of as a difference of
// two nearly equal residuals).
template <typename T, bool EDGE, bool ABS>
struct Pipe {
    static constexpr int V = Vec<T>::N;
    static constexpr int NP = ABS ? NPART_L1 : NPART;
    static constexpr int IL1 = ABS ? 1 : 6, IL2 = ABS ? 2 : 7;  // sum |u|, sum u^2
    TileCtx<T> c;
    T UX[4][V];                              // u^x_n
    T UT[2][V], PH[2][V], SV[2][V], RV[2][V];  // u^t_n, phi_{n-1}, s, R
    T PHN[2][V], AN[2][V];   // phi_n and A_n = div u_n + s
    T DX[2][V], DT[2][V];    // u_{n+1} - u_n
    T A1[2][V], B1[2][V];    // A_{n+1}, B_{n+1} (one row behind)
    double acc[NP];

    __device__ explicit Pipe(const TileCtx<T>& ctx) : c(ctx)
    {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            zero(PHN[b]); zero(AN[b]); zero(DX[b]); zero(DT[b]); zero(A1[b]); zero(B1[b]);
        }
#pragma unroll
        for (int m = 0; m < NP; ++m) acc[m] = 0.0;
    }

    // byte offset of row i for loads (rows past the grid fall out of range)
    __device__ __forceinline__ uint32_t lrow(int i) const { return c.vb_ld + (uint32_t)i * c.row_bytes; }

    // The prefetches run ahead of the march; rows the tile never reads (u^x past
    // ilast + 1, the other fields past ilast) go out of range instead of to memory.
    __device__ __forceinline__ void load_x(int i, T (&ux)[V])
    {
        bload(c.uxi, i <= c.ilast + 1 ? lrow(i) : OOB, ux);
    }
    __device__ __forceinline__ void load_rest(int i, T (&ut)[V], T (&ph)[V], T (&sv)[V], T (&rv)[V])
    {
        const uint32_t o = i <= c.ilast ? lrow(i) : OOB;
        bload(c.uti, o, ut);
        bload(c.phi_i, o, ph);
        bload(c.si, o, sv);
        bload(c.ri, o, rv);
    }

    __device__ __forceinline__ void start()
    {
        load_x(c.ibeg, UX[0]);
        load_x(c.ibeg + 1, UX[1]);
        load_x(c.ibeg + 2, UX[2]);
        load_rest(c.ibeg, UT[0], PH[0], SV[0], RV[0]);
    }

    // residual of the new flux on row im and its contribution to the products;
    // DXf: flux change of row im + 1 (zeros past the grid), P: set of row im
    template <int P>
    __device__ __forceinline__ void close_row(int im, const T (&DXf)[V], bool has_next)
    {
        constexpr int Q = P ^ 1;
        T b[V];
        const T dt_next = lane_next(DT[P][0]);
        T zero_add[V];
        zero(zero_add);
        div_row<T, EDGE>(c, has_next, im > 0, DX[P], DXf, DT[P], dt_next, zero_add, b);
        T a[V];
#pragma unroll
        for (int k = 0; k < V; ++k) a[k] = AN[P][k] + b[k];
        const T a_prev = lane_prev(a[V - 1]);
        const T b_prev = lane_prev(b[V - 1]);
        if (im >= c.r0 && im < c.rend && c.lane_out) {
            const bool xg = im > 0;
#pragma unroll
            for (int k = 0; k < V; ++k) {
                if (EDGE && !c.inb[k]) continue;
                const T ap = (k > 0) ? a[(k + V - 1) % V] : a_prev;
                const T bp = (k > 0) ? b[(k + V - 1) % V] : b_prev;
                const double gax = xg ? double((a[k] - A1[Q][k]) * c.idx) : 0.0;
                const double gbx = xg ? double((b[k] - B1[Q][k]) * c.idx) : 0.0;
                double gat = double((a[k] - ap) * c.idt);
                double gbt = double((b[k] - bp) * c.idt);
                if constexpr (EDGE) {
                    gat = c.jgt0[k] ? gat : 0.0;
                    gbt = c.jgt0[k] ? gbt : 0.0;
                }
                const double av = double(a[k]), bv = double(b[k]);
                if constexpr (ABS) {
                    acc_cell<true>(acc, c.thm, av, bv, gat, gbt);
                    acc_xgrad<true>(acc, c.thm, gax, gbx);
                } else {
                    acc[0] = fma(av, av, acc[0]);
                    acc[1] = fma(av, bv, acc[1]);
                    acc[2] = fma(bv, bv, acc[2]);
                    acc[3] = fma(gax, gax, fma(gat, gat, acc[3]));
                    acc[4] = fma(gax, gbx, fma(gat, gbt, acc[4]));
                    acc[5] = fma(gbx, gbx, fma(gbt, gbt, acc[5]));
                }
            }
        }
#pragma unroll
        for (int k = 0; k < V; ++k) {
            A1[P][k] = a[k];
            B1[P][k] = b[k];
        }
    }

    // step on grid row i (i < nr); S: position of row i mod 4
    template <int S, bool PROX>
    __device__ __forceinline__ void step(int i)
    {
        constexpr int P = S & 1, Q = P ^ 1;
        constexpr int X0 = S, X1 = (S + 1) & 3, X3 = (S + 3) & 3;
        const bool own_row = (i >= c.r0) && (i < c.rend);
        // store offset: rows outside the strip and halo lanes fall out of range
        const uint32_t so = c.vb_st + (own_row ? (uint32_t)i * c.row_bytes : OOB);
        const bool has_prev = i > 0;
        load_x(i + 3, UX[X3]);  // row i - 1's registers
        load_rest(i + 1, UT[Q], PH[Q], SV[Q], RV[Q]);

        // (1) residual of the current flux: A_n = div u_n + s on row i
        div_row<T, EDGE>(c, i + 1 < c.nr, has_prev, UX[X0], UX[X1], UT[P],
                         lane_next(UT[P][0]), SV[P], AN[P]);
        // (2) dual step: phi_n = phi_{n-1} + beta (A_n + theta (A_n - R))
#pragma unroll
        for (int k = 0; k < V; ++k)
            PHN[P][k] = fma(c.beta, fma(c.theta, AN[P][k] - RV[P][k], AN[P][k]), PH[P][k]);
        {
            T w[V];
#pragma unroll
            for (int k = 0; k < V; ++k) w[k] = (!EDGE || c.inb[k]) ? PHN[P][k] : T(0);
            bstore(c.phio, so, w);
            if constexpr (PROX) {
#pragma unroll
                for (int k = 0; k < V; ++k) w[k] = (!EDGE || c.inb[k]) ? AN[P][k] : T(0);
                bstore(c.ro, so, w);
            }
        }
        if constexpr (PROX) {
            // (3) primal update with the backward-difference gradient of phi_n
            const T ph_prev = lane_prev(PHN[P][V - 1]);
            const T wgx = has_prev ? c.idx : T(0);
            T u1x[V], u1t[V];
            T l1 = T(0), l2 = T(0);
#pragma unroll
            for (int k = 0; k < V; ++k) {
                const T gx = (PHN[P][k] - PHN[Q][k]) * wgx;
                const T pprev = (k > 0) ? PHN[P][(k + V - 1) % V] : ph_prev;
                T gt = (PHN[P][k] - pprev) * c.idt;
                if constexpr (EDGE) gt = c.jgt0[k] ? gt : T(0);
                u1x[k] = shrink_scaled(fma(c.alpha, gx, UX[X0][k]), c.alpha, c.inv);
                u1t[k] = shrink_scaled(fma(c.alpha, gt, UT[P][k]), c.alpha, c.inv);
                DX[P][k] = u1x[k] - UX[X0][k];
                DT[P][k] = u1t[k] - UT[P][k];
                if (!EDGE || c.inb[k]) {
                    l1 += fabs(u1x[k]) + fabs(u1t[k]);
                    l2 = fma(u1x[k], u1x[k], fma(u1t[k], u1t[k], l2));
                }
            }
            {
                T w[V];
#pragma unroll
                for (int k = 0; k < V; ++k) w[k] = (!EDGE || c.inb[k]) ? u1x[k] : T(0);
                bstore(c.uxo, so, w);
#pragma unroll
                for (int k = 0; k < V; ++k) w[k] = (!EDGE || c.inb[k]) ? u1t[k] : T(0);
                bstore(c.uto, so, w);
            }
            if (own_row && c.lane_out) {
                acc[IL1] += double(l1);
                acc[IL2] += double(l2);
            }
            // (4) residual of the new flux on row i - 1
            if (i > c.ibeg) close_row<Q>(i - 1, DX[P], true);
        }
    }

    // the march over the tile's rows: grid rows [ibeg, iend) -- through ilast when
    // it is a grid row (it closes the strip's last own row), else through nr - 1
    // followed by the virtual row nr
    template <bool PROX>
    __device__ __forceinline__ void run()
    {
        const int iend = min(c.ilast + 1, c.nr);
        int i = c.ibeg;
        for (; i + 3 < iend; i += 4) {
            step<0, PROX>(i);
            step<1, PROX>(i + 1);
            step<2, PROX>(i + 2);
            step<3, PROX>(i + 3);
        }
        int last_set = 1;  // parity set of the last row stepped
        if (i < iend) {
            step<0, PROX>(i++);
            last_set = 0;
            if (i < iend) {
                step<1, PROX>(i++);
                last_set = 1;
                if (i < iend) {
                    step<2, PROX>(i++);
                    last_set = 0;
                }
            }
        }
        if constexpr (PROX) {
            if (c.ilast == c.nr) {
                // bring the last row into set 0 by value (selecting between register
                // sets by a runtime index would push them out to scratch memory)
                const bool swap = last_set == 1;
#pragma unroll
                for (int k = 0; k < V; ++k) {
                    swap2(swap, DX[0][k], DX[1][k]);
                    swap2(swap, DT[0][k], DT[1][k]);
                    swap2(swap, AN[0][k], AN[1][k]);
                    swap2(swap, A1[0][k], A1[1][k]);
                    swap2(swap, B1[0][k], B1[1][k]);
                }
                T zero_row[V];
                zero(zero_row);
                close_row<0>(c.nr - 1, zero_row, false);
            }
        }
    }
};

// The upward march, used on odd strips.  A tile shares its halo rows with the
// strips above and below; if every tile marched down, the two reads of a shared
// row would be a whole tile lifetime apart and the second would miss the L2.  With
// even strips marching down and odd strips up, both tiles at every strip boundary
// read the shared rows near the start of their march, or both near the end.
// The per-cell arithmetic is that of the downward march, with the same operands in
// the same order, so the fields are bitwise the same; only the order in which the
// cells are summed into the partials differs.  Marching up, the flux update of
// row i + 1 needs phi_n of the row above it, row i, so it runs one row behind the
// dual step, and the residual of the new flux one row behind that:
//   step i: A_n and phi_n of row i, u_{n+1} of row i + 1, residual of row i + 1.
// The x-gradient of the new residual at row i + 1 pairs it with row i + 2, closed
// one step earlier.  The march ends at a virtual row -1 when it reaches the top of
// the grid, so that row 0 gets its flux update and residual (nothing is loaded or
// stored for row -1, and its gradient weight is zero).
template <typename T, bool EDGE, bool ABS>
struct PipeUp {
    static constexpr int V = Vec<T>::N;
    static constexpr int NP = ABS ? NPART_L1 : NPART;
    static constexpr int IL1 = ABS ? 1 : 6, IL2 = ABS ? 2 : 7;
    TileCtx<T> c;
    int ib;                                // bottom row of the march
    T UX[4][V], UT[4][V];                  // u_n: row i in set S, i + 1 in S + 3
    T PH[2][V], SV[2][V], RV[2][V];        // phi_{n-1}, s, R: row i (P), row i - 1 (Q)
    T PHN[2][V], AN[2][V];                 // phi_n, A_n: row i (P), row i + 1 (Q)
    T DX[2][V], DT[2][V];                  // u_{n+1} - u_n: row i + 1 (P), row i + 2 (Q)
    T A1[V], B1[V];                        // A_{n+1}, B_{n+1} of the last residual row
    double acc[NP];

    __device__ explicit PipeUp(const TileCtx<T>& ctx) : c(ctx)
    {
        ib = min(c.ilast, c.nr - 1);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            zero(PHN[b]); zero(AN[b]); zero(DX[b]); zero(DT[b]);
        }
        zero(A1);
        zero(B1);
#pragma unroll
        for (int m = 0; m < NP; ++m) acc[m] = 0.0;
    }

    __device__ __forceinline__ uint32_t lrow(int i) const { return c.vb_ld + (uint32_t)i * c.row_bytes; }

    // rows above the march's top row are never read: they go out of range
    __device__ __forceinline__ void load_u(int i, T (&ux)[V], T (&ut)[V])
    {
        const uint32_t o = i >= c.ibeg ? lrow(i) : OOB;
        bload(c.uxi, o, ux);
        bload(c.uti, o, ut);
    }
    __device__ __forceinline__ void load_rest(int i, T (&ph)[V], T (&sv)[V], T (&rv)[V])
    {
        const uint32_t o = i >= c.ibeg ? lrow(i) : OOB;
        bload(c.phi_i, o, ph);
        bload(c.si, o, sv);
        bload(c.ri, o, rv);
    }

    __device__ __forceinline__ void start()
    {
        load_u(ib, UX[0], UT[0]);
        // u^x of the row below the march (zeros past the grid); u^t there is unused
        bload(c.uxi, lrow(ib + 1), UX[3]);
        zero(UT[3]);
        load_u(ib - 1, UX[1], UT[1]);
        load_rest(ib, PH[0], SV[0], RV[0]);
    }

    // residual of the new flux on row im: its products, and the x-gradient products
    // of row im + 1 (whose residual is in A1, B1)
    template <int P>
    __device__ __forceinline__ void close_row(int im)
    {
        constexpr int Q = P ^ 1;
        T b[V];
        const T dt_next = lane_next(DT[P][0]);
        T zero_add[V];
        zero(zero_add);
        div_row<T, EDGE>(c, im + 1 < c.nr, im > 0, DX[P], DX[Q], DT[P], dt_next, zero_add, b);
        T a[V];
#pragma unroll
        for (int k = 0; k < V; ++k) a[k] = AN[Q][k] + b[k];
        const T a_prev = lane_prev(a[V - 1]);
        const T b_prev = lane_prev(b[V - 1]);
        const bool own = im >= c.r0 && im < c.rend;
        const bool own_below = im + 1 >= c.r0 && im + 1 < c.rend;
        if ((own || own_below) && c.lane_out) {
#pragma unroll
            for (int k = 0; k < V; ++k) {
                if (EDGE && !c.inb[k]) continue;
                if (own) {
                    const T ap = (k > 0) ? a[(k + V - 1) % V] : a_prev;
                    const T bp = (k > 0) ? b[(k + V - 1) % V] : b_prev;
                    double gat = double((a[k] - ap) * c.idt);
                    double gbt = double((b[k] - bp) * c.idt);
                    if constexpr (EDGE) {
                        gat = c.jgt0[k] ? gat : 0.0;
                        gbt = c.jgt0[k] ? gbt : 0.0;
                    }
                    acc_cell<ABS>(acc, c.thm, double(a[k]), double(b[k]), gat, gbt);
                }
                if (own_below) {
                    const double gax = double((A1[k] - a[k]) * c.idx);
                    const double gbx = double((B1[k] - b[k]) * c.idx);
                    acc_xgrad<ABS>(acc, c.thm, gax, gbx);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < V; ++k) {
            A1[k] = a[k];
            B1[k] = b[k];
        }
    }

    // step on row i (ibeg - 1 <= i <= ib); S = (ib - i) mod 4; HEAD: the first
    // step, which has no row below it to update
    template <int S, bool HEAD>
    __device__ __forceinline__ void step(int i)
    {
        constexpr int P = S & 1, Q = P ^ 1;
        constexpr int X0 = S, X2 = (S + 2) & 3, X3 = (S + 3) & 3;
        const bool own_i = (i >= c.r0) && (i < c.rend);
        const uint32_t so_i = c.vb_st + (own_i ? (uint32_t)i * c.row_bytes : OOB);
        load_u(i - 2, UX[X2], UT[X2]);
        load_rest(i - 1, PH[Q], SV[Q], RV[Q]);

        // (1) residual of the current flux: A_n = div u_n + s on row i
        div_row<T, EDGE>(c, i + 1 < c.nr, i > 0, UX[X0], UX[X3], UT[X0],
                         lane_next(UT[X0][0]), SV[P], AN[P]);
        // (2) dual step on row i
#pragma unroll
        for (int k = 0; k < V; ++k)
            PHN[P][k] = fma(c.beta, fma(c.theta, AN[P][k] - RV[P][k], AN[P][k]), PH[P][k]);
        {
            T w[V];
#pragma unroll
            for (int k = 0; k < V; ++k) w[k] = (!EDGE || c.inb[k]) ? PHN[P][k] : T(0);
            bstore(c.phio, so_i, w);
#pragma unroll
            for (int k = 0; k < V; ++k) w[k] = (!EDGE || c.inb[k]) ? AN[P][k] : T(0);
            bstore(c.ro, so_i, w);
        }
        if constexpr (!HEAD) {
            // (3) primal update of row i + 1 with phi_n of rows i + 1 and i
            const int in = i + 1;
            const bool own_n = (in >= c.r0) && (in < c.rend);
            const uint32_t so_n = c.vb_st + (own_n ? (uint32_t)in * c.row_bytes : OOB);
            const T ph_prev = lane_prev(PHN[Q][V - 1]);
            const T wgx = in > 0 ? c.idx : T(0);
            T u1x[V], u1t[V];
            T l1 = T(0), l2 = T(0);
#pragma unroll
            for (int k = 0; k < V; ++k) {
                const T gx = (PHN[Q][k] - PHN[P][k]) * wgx;
                const T pprev = (k > 0) ? PHN[Q][(k + V - 1) % V] : ph_prev;
                T gt = (PHN[Q][k] - pprev) * c.idt;
                if constexpr (EDGE) gt = c.jgt0[k] ? gt : T(0);
                u1x[k] = shrink_scaled(fma(c.alpha, gx, UX[X3][k]), c.alpha, c.inv);
                u1t[k] = shrink_scaled(fma(c.alpha, gt, UT[X3][k]), c.alpha, c.inv);
                DX[P][k] = u1x[k] - UX[X3][k];
                DT[P][k] = u1t[k] - UT[X3][k];
                if (!EDGE || c.inb[k]) {
                    l1 += fabs(u1x[k]) + fabs(u1t[k]);
                    l2 = fma(u1x[k], u1x[k], fma(u1t[k], u1t[k], l2));
                }
            }
            {
                T w[V];
#pragma unroll
                for (int k = 0; k < V; ++k) w[k] = (!EDGE || c.inb[k]) ? u1x[k] : T(0);
                bstore(c.uxo, so_n, w);
#pragma unroll
                for (int k = 0; k < V; ++k) w[k] = (!EDGE || c.inb[k]) ? u1t[k] : T(0);
                bstore(c.uto, so_n, w);
            }
            if (own_n && c.lane_out) {
                acc[IL1] += double(l1);
                acc[IL2] += double(l2);
            }
            // (4) residual of the new flux on row i + 1
            close_row<P>(in);
        }
    }

    // the march from row ib up to ibeg (to the virtual row -1 at the top of the grid)
    __device__ __forceinline__ void run()
    {
        const int itop = c.ibeg > 0 ? c.ibeg : -1;
        int i = ib;
        step<0, true>(i--);
        for (; i - 3 >= itop; i -= 4) {
            step<1, false>(i);
            step<2, false>(i - 1);
            step<3, false>(i - 2);
            step<0, false>(i - 3);
        }
        if (i >= itop) {
            step<1, false>(i--);
            if (i >= itop) {
                step<2, false>(i--);
                if (i >= itop) step<3, false>(i--);
            }
        }
    }
};

// Evaluation sweep of the l1 linesearch, for a gather none of whose NL1 candidates
// passed: recompute, exactly as the previous sweep formed them, the residual
// A_n = A_{n-1} + div(u_n - u_{n-1}) and B_n = div(u_n - u_{n-1}) from u_n (the
// input buffers) and u_{n-1} (the output buffers, which this sweep leaves alone),
// and sum the test for the next NL1 candidates together with <A,A>, sum |u_n| and
// sum u_n^2.  Rare, so one plain row at a time; no field is written.
template <typename T>
__device__ void eval_tile(const TileCtx<T>& c, double (&acc)[NPART_L1])
{
    constexpr int V = Vec<T>::N;
#pragma unroll
    for (int m = 0; m < NPART_L1; ++m) acc[m] = 0.0;
    T a_up[V], b_up[V];  // A_n, B_n of the row above
    zero(a_up);
    zero(b_up);
    T zero_add[V];
    zero(zero_add);
    for (int im = max(c.r0 - 1, 0); im < c.rend; ++im) {
        const uint32_t o0 = c.vb_ld + (uint32_t)im * c.row_bytes;
        const uint32_t o1 = o0 + c.row_bytes;  // row im + 1: out of range past the grid
        T nx0[V], nt0[V], nx1[V], ox0[V], ot0[V], ox1[V], sv[V];
        bload(c.uxi, o0, nx0);
        bload(c.uti, o0, nt0);
        bload(c.uxi, o1, nx1);
        bload(c.uxo, o0, ox0);
        bload(c.uto, o0, ot0);
        bload(c.uxo, o1, ox1);
        bload(c.si, o0, sv);
        T an[V], dx0[V], dx1[V], dt0[V], b[V], a[V];
        div_row<T, true>(c, im + 1 < c.nr, im > 0, ox0, ox1, ot0, lane_next(ot0[0]), sv, an);
#pragma unroll
        for (int k = 0; k < V; ++k) {
            dx0[k] = nx0[k] - ox0[k];
            dx1[k] = nx1[k] - ox1[k];
            dt0[k] = nt0[k] - ot0[k];
        }
        div_row<T, true>(c, im + 1 < c.nr, im > 0, dx0, dx1, dt0, lane_next(dt0[0]), zero_add, b);
#pragma unroll
        for (int k = 0; k < V; ++k) a[k] = an[k] + b[k];
        const T a_prev = lane_prev(a[V - 1]);
        const T b_prev = lane_prev(b[V - 1]);
        if (im >= c.r0 && c.lane_out) {
            const bool xg = im > 0;
            T l1 = T(0), l2 = T(0);
#pragma unroll
            for (int k = 0; k < V; ++k) {
                if (!c.inb[k]) continue;
                const T ap = (k > 0) ? a[(k + V - 1) % V] : a_prev;
                const T bp = (k > 0) ? b[(k + V - 1) % V] : b_prev;
                const double gat = c.jgt0[k] ? double((a[k] - ap) * c.idt) : 0.0;
                const double gbt = c.jgt0[k] ? double((b[k] - bp) * c.idt) : 0.0;
                const double gax = xg ? double((a[k] - a_up[k]) * c.idx) : 0.0;
                const double gbx = xg ? double((b[k] - b_up[k]) * c.idx) : 0.0;
                acc_cell<true>(acc, c.thm, double(a[k]), double(b[k]), gat, gbt);
                acc_xgrad<true>(acc, c.thm, gax, gbx);
                l1 += fabs(nx0[k]) + fabs(nt0[k]);
                l2 = fma(nx0[k], nx0[k], fma(nt0[k], nt0[k], l2));
            }
            acc[1] += double(l1);
            acc[2] += double(l2);
        }
#pragma unroll
        for (int k = 0; k < V; ++k) {
            a_up[k] = a[k];
            b_up[k] = b[k];
        }
    }
}

// One tile: set up the lane's view, put the first rows in flight, then take the
// gather's decision (which reduces the previous sweep's partials) while they load.
// UP: the tile marches up its rows (odd strips, see PipeUp); the last sweep of a
// gather (dual step only) always marches down.  ABS: l1 linesearch test.
// p: sweep parity (partials, scalar state); pb: buffer parity of the fields.
template <typename T, bool EDGE, bool UP, bool ABS>
__device__ void sweep_tile(const SweepArgs<T>& a, const Tile& tl, const GatherMeta& gm, int p, int pb,
                           int w, double* red)
{
    constexpr int V = Vec<T>::N;
    constexpr int NP = ABS ? NPART_L1 : NPART;
    const int lane = threadIdx.x & (WAVE - 1);
    const int q = p ^ 1, qb = pb ^ 1;
    TileCtx<T> c;
    c.nr = gm.nr;
    c.ld = gm.ld;
    const int nt = gm.nt;
    c.r0 = tl.r0;
    c.rend = min(tl.r0 + gm.rows, gm.nr);
    c.ibeg = max(tl.r0 - 2, 0);
    c.ilast = min(tl.r0 + gm.rows, gm.nr);  // == nr: the virtual row closes the last strip
    const int j0 = tl.c0 - V + V * lane;
    const bool lane_load = (lane <= HALO_LANE_R) && (j0 >= 0) && (j0 < nt);
    c.lane_out = (lane >= 1) && (lane <= OUT_LANES) && lane_load;
#pragma unroll
    for (int k = 0; k < V; ++k) {
        const int j = j0 + k;
        c.inb[k] = (j >= 0) && (j < nt);
        c.jgt0[k] = j > 0;
        c.jlt[k] = j + 1 < nt;
    }
    c.idx = T(1.0 / gm.dx);
    c.idt = T(1.0 / gm.dt);
    c.row_bytes = (uint32_t)(gm.ld * sizeof(T));
    c.vb_ld = lane_load ? (uint32_t)(j0 * (int)sizeof(T)) : OOB;
    c.vb_st = c.lane_out ? (uint32_t)(j0 * (int)sizeof(T)) : OOB;
    const int bytes = (int)((int64_t)gm.nr * gm.ld * sizeof(T));
    auto rs = [&](const T* f) {
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(f + gm.poff), 0, bytes, 0x00020000);
    };
    c.uxi = rs(a.ux[pb]);
    c.uti = rs(a.ut[pb]);
    c.phi_i = rs(a.phi[pb]);
    c.ri = rs(a.R[pb]);
    c.si = rs(a.s);
    c.uxo = rs(a.ux[qb]);
    c.uto = rs(a.ut[qb]);
    c.phio = rs(a.phi[qb]);
    c.ro = rs(a.R[qb]);

    using Pipeline = typename std::conditional<UP, PipeUp<T, EDGE, ABS>, Pipe<T, EDGE, ABS>>::type;
    Pipeline P(c);
    P.start();
    const Decision d = decide<T, ABS>(a, p, tl.g, gm, tl.slot == gm.tile_base, pb, w, red);
    if (!d.run) return;
    P.c.beta = T(d.beta);
    P.c.theta = T(d.theta);
    P.c.alpha = T(d.alpha);
    P.c.inv = T(1.0 / (1.0 + a.sc.eps * d.alpha));
    if constexpr (ABS) {
        // the candidate thetas of the next decision, as it will form them
        double alpha = uniform_d(d.cand0);
        const double ref = uniform_d(d.cand_ref);
#pragma unroll
        for (int m = 0; m < NL1; ++m) {
            P.c.thm[m] = alpha / ref;
            alpha *= a.sc.xi;
        }
    }
    double* __restrict__ dst = a.part[q] + (int64_t)tl.slot * NP;
    if constexpr (ABS) {
        if (d.eval) {
            double acc[NPART_L1];
            eval_tile<T>(P.c, acc);
#pragma unroll
            for (int m = 0; m < NPART_L1; ++m) acc[m] = wave_sum(acc[m]);
            if (lane == 0) {
#pragma unroll
                for (int m = 0; m < NPART_L1; ++m) dst[m] = acc[m];
            }
            return;
        }
    }
    if (d.prox) {
        if constexpr (UP) P.run();
        else P.template run<true>();
#pragma unroll
        for (int m = 0; m < NP; ++m) P.acc[m] = wave_sum(P.acc[m]);
        if (lane == 0) {
#pragma unroll
            for (int m = 0; m < NP; ++m) dst[m] = P.acc[m];
        }
    } else if constexpr (UP) {
        Pipe<T, EDGE, ABS> D(P.c);
        D.start();
        D.template run<false>();
    } else {
        P.template run<false>();
    }
}

template <typename T, bool ABS>
__global__ __launch_bounds__(256) void k_sweep(SweepArgs<T> a, int parity)
{
    constexpr int V = Vec<T>::N;
    constexpr int NP = ABS ? NPART_L1 : NPART;
    constexpr int WPB = 256 / WAVE;  // waves per block (4: the quarters of the record sums)
    static_assert(WPB == 4, "the decision sums are split in four quarters");
    __shared__ double red[WPB * NP];
    const int w = uniform((int)threadIdx.x / WAVE);
    const int first = uniform(xcd_logical_block() * WPB);  // table entry of wave 0
    const int tid = first + w;
    if (tid >= a.ntiles) return;
    // When every real entry of this block belongs to one running gather past its
    // first sweep, its four waves (padding entries included) share the work of that
    // gather's decision sums; every wave of such a block reaches the one barrier in
    // decision_sums.  Each wave works this out from the same four entries.
    int gb = -1;
    bool split = first + WPB <= a.ntiles;
    for (int k = 0; k < WPB && split; ++k) {
        const int gk = uniform(a.tiles[first + k].g);
        if (gk < 0) continue;
        if (gb < 0) gb = gk;
        else if (gk != gb) split = false;
    }
    if (gb < 0) split = false;
    if (split) {
        const GState* sb = a.gst[parity] + gb;
        split = uniform(sb->status) == ST_RUNNING && uniform(sb->started) != 0;
    }
    const Tile tl = a.tiles[tid];
    const int g = uniform(tl.g);
    if (g < 0) {
        // padding entry: only its quarter of the block gather's decision sums
        if (split) {
            const GatherMeta mb = a.meta[gb];
            double s[NP];
            decision_sums<NP>(a.part[parity] + (int64_t)mb.tile_base * NP, mb.ntiles, w, red, s);
        }
        return;
    }
    double* const xred = split ? red : nullptr;
    const GatherMeta gm = a.meta[g];
    const GState* gs = a.gst[parity] + g;
    if (gs->status != ST_RUNNING) {
        // finished gather: only carry its state to the other parity
        if (tl.slot == gm.tile_base && (threadIdx.x & (WAVE - 1)) == 0)
            a.gst[parity ^ 1][g] = *gs;
        return;
    }
    const int pb = uniform(parity ^ gs->flip);
    // tiles whose loaded lanes (0..OUT_LANES + 1) all sit strictly inside (0, nt - 1)
    // need no time-boundary masks
    const bool edge = (tl.c0 - V < 1) || (tl.c0 + HALO_LANE_R * V > gm.nt - 1);
    // odd strips march up
    const bool up = ((tl.r0 / gm.rows) & 1) != 0;
    if (edge) {
        if (up) sweep_tile<T, true, true, ABS>(a, tl, gm, parity, pb, w, xred);
        else sweep_tile<T, true, false, ABS>(a, tl, gm, parity, pb, w, xred);
    } else {
        if (up) sweep_tile<T, false, true, ABS>(a, tl, gm, parity, pb, w, xred);
        else sweep_tile<T, false, false, ABS>(a, tl, gm, parity, pb, w, xred);
    }
}

// ======================================================================================
// Plain PDHG with the fixed steps alpha_1, beta_1 = delta alpha_1 and theta = 1 (the
// primal and dual updates of Section 2.2 before the linesearch is introduced), two
// iterations per HBM pass.  With no linesearch nothing global sits between two
// iterations, so one sweep takes (u_k, phi_k) to (u_{k+2}, phi_{k+2}):
//   u_{k+1}   = shrink(u_k + alpha grad phi_k, alpha) / (1 + eps alpha)        (P1)
//   phi_{k+1} = phi_k + beta (A_{k+1} + (A_{k+1} - A_k)),  A_m = div u_m + s     (D1)
//   u_{k+2}   = shrink(u_{k+1} + alpha grad phi_{k+1}, alpha) / (1 + eps alpha) (P2)
//   phi_{k+2} = phi_{k+1} + beta (A_{k+2} + (A_{k+2} - A_{k+1}))              (D2)
// (A + (A - A') = div(2 u - u') + s: the dual step at ubar = 2 u_{m+1} - u_m.)  The
// state is (u, phi) only: each A is recomputed from its flux, with the operands and
// operations of the one-iteration sweep (which stores A_k as R), so the fields are
// bitwise those of that sweep with fixed steps.  A sweep reads u, phi, s (16 bytes per
// cell in FP32) and writes u, phi (12 bytes) for two iterations, against 36 bytes per
// iteration for the linesearch sweep.
//
// The dependency cone grows by one row and one sample per stage: a tile loads two
// rows above and two below its own rows, and its halo lanes (0 and 57, four samples
// each) cover the two samples either way.  On even strips the wave marches down; at
// step i (row i just loaded) it forms P1 of row i, A_k, A_{k+1} and D1 of row i - 1,
// P2 of row i - 1, then A_{k+2} and D2 of row i - 2.  Loaded rows sit in register sets
// indexed by row mod 4 (the next row loads into the set of row i - 3), computed rows
// in sets indexed by row mod 2; the loop is unrolled by four so every index is static.
// Odd strips march up (Pipe2Up), so that neighbouring strips read their shared rows
// together.
// ======================================================================================

struct Decision2 {
    double alpha, beta;
    int steps;  // PDHG iterations this sweep applies to the gather (0: none)
};

// The gather's decision at the start of a sweep of K iterations: the stop rule on the
// sums of the previous sweep (which describe u_k, the flux this sweep reads), then how
// many iterations this sweep runs: K, or fewer to bring a count that is not a
// multiple of K (a resumed checkpoint) back to one, or to end at max_iter.  Checks
// fall on multiples of K.
template <typename T, int K>
__device__ Decision2 decide_fixedk(const SweepArgs<T>& a, int p, int g, const GatherMeta& gm, bool writer,
                                   int pb, int w, double* red)
{
    const GState* __restrict__ sin = a.gst[p] + g;
    GState* __restrict__ sout = a.gst[p ^ 1] + g;
    GState st = *sin;
    const SolveScalars& sc = a.sc;
    Decision2 d;
    d.alpha = st.alpha;
    d.beta = sc.delta * st.alpha;
    d.steps = 0;
    const int lane = threadIdx.x & (WAVE - 1);
    if (st.status != ST_RUNNING) {
        if (writer && lane == 0) *sout = st;
        return d;
    }
    int status = ST_RUNNING;
    if (st.started) {
        double q[NPART];
        decision_sums<NPART>(a.part[p] + (int64_t)gm.tile_base * NPART, gm.ntiles, w, red, q);
        const double aa = q[0], l1 = q[6], l2 = q[7];
        if (!(isfinite(aa) && isfinite(l1) && isfinite(l2))) {
            status = ST_NONFINITE;
        } else {
            st.rel_res = sqrt(aa) / st.snorm;
            st.emd = gm.cm * (l1 + 0.5 * sc.eps * l2);
            st.transport = gm.cm * l1;
            if (sc.hist && writer && lane == 0 && st.iters % sc.check_every == 0)
                sc.hist[(int64_t)g * sc.hist_cap + (st.iters / sc.check_every - 1) % sc.hist_cap] = st.rel_res;
            if (st.iters % sc.check_every == 0 && st.rel_res <= sc.tol_res) status = ST_CONVERGED;
            else if (st.iters >= sc.max_iter) status = ST_MAX_ITER;
        }
    }
    if (status != ST_RUNNING) {
        // u_k and phi_k are this sweep's inputs
        st.ubuf = pb;
        st.phibuf = pb;
        st.status = status;
        if (writer && lane == 0) {
            *sout = st;
            atomicAdd(a.done, 1);
        }
        return d;
    }
    st.started = 1;
    int steps = K - st.iters % K;
    if (steps > sc.max_iter - st.iters) steps = max(sc.max_iter - st.iters, 1);
    st.iters += steps;
    st.ubuf = pb ^ 1;
    st.phibuf = pb ^ 1;
    if (writer && lane == 0) *sout = st;
    d.steps = steps;
    return d;
}

template <typename T, bool EDGE>
struct Pipe2 {
    static constexpr int V = Vec<T>::N;
    TileCtx<T> c;
    int iend;                                // last step (row index; past nr: virtual rows)
    T LX[4][V], LT[4][V], LP[4][V], LS[4][V];  // u^x_k, u^t_k, phi_k, s of loaded rows, by row mod 4
    T P1X[2][V], P1T[2][V];                  // u_{k+1}: rows i (set i & 1) and i - 1
    T A1[2][V], D1[2][V];                    // A_{k+1}, phi_{k+1}: rows i - 1 and i - 2
    T P2X[2][V], P2T[2][V];                  // u_{k+2}: rows i - 1 and i - 2
    double aa, l1, l2;

    __device__ explicit Pipe2(const TileCtx<T>& ctx) : c(ctx)
    {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            zero(LX[b]); zero(LT[b]); zero(LP[b]); zero(LS[b]);
        }
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            zero(P1X[b]); zero(P1T[b]); zero(A1[b]); zero(D1[b]); zero(P2X[b]); zero(P2T[b]);
        }
        aa = l1 = l2 = 0.0;
    }

    __device__ __forceinline__ void load(int i, T (&ux)[V], T (&ut)[V], T (&ph)[V], T (&sv)[V])
    {
        const uint32_t o = i <= c.ilast ? c.vb_ld + (uint32_t)i * c.row_bytes : OOB;
        bload(c.uxi, o, ux);
        bload(c.uti, o, ut);
        bload(c.phi_i, o, ph);
        bload(c.si, o, sv);
    }

    __device__ __forceinline__ bool own(int m) const { return m >= c.r0 && m < c.rend; }
    __device__ __forceinline__ uint32_t store_off(int m) const
    {
        return c.vb_st + (own(m) ? (uint32_t)m * c.row_bytes : OOB);
    }

    // the shrink step of the primal update on one row: u' = prox(u + alpha grad phi),
    // grad the backward difference (phi of the row above: pu, weight wgx)
    __device__ __forceinline__ void prox_row(const T (&ux)[V], const T (&ut)[V], const T (&ph)[V],
                                             const T (&pu)[V], bool has_prev, T (&ox)[V], T (&ot)[V]) const
    {
        const T ph_prev = lane_prev(ph[V - 1]);
        const T wgx = has_prev ? c.idx : T(0);
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const T gx = (ph[k] - pu[k]) * wgx;
            const T pprev = (k > 0) ? ph[(k + V - 1) % V] : ph_prev;
            T gt = (ph[k] - pprev) * c.idt;
            if constexpr (EDGE) gt = c.jgt0[k] ? gt : T(0);
            ox[k] = shrink_scaled(fma(c.alpha, gx, ux[k]), c.alpha, c.inv);
            ot[k] = shrink_scaled(fma(c.alpha, gt, ut[k]), c.alpha, c.inv);
        }
    }

    __device__ __forceinline__ void dual_row(const T (&an)[V], const T (&r)[V], const T (&ph)[V], T (&out)[V]) const
    {
#pragma unroll
        for (int k = 0; k < V; ++k) out[k] = fma(c.beta, fma(c.theta, an[k] - r[k], an[k]), ph[k]);
    }

    __device__ __forceinline__ void store(__amdgpu_buffer_rsrc_t r, uint32_t off, const T (&x)[V]) const
    {
        T w[V];
#pragma unroll
        for (int k = 0; k < V; ++k) w[k] = (!EDGE || c.inb[k]) ? x[k] : T(0);
        bstore(r, off, w);
    }

    // sums for the stop rule: sum |u|, sum u^2 of a flux row, <A, A> of a residual row
    __device__ __forceinline__ void sum_flux(int m, const T (&ux)[V], const T (&ut)[V])
    {
        if (!(own(m) && c.lane_out)) return;
        T s1 = T(0), s2 = T(0);
#pragma unroll
        for (int k = 0; k < V; ++k) {
            if (!EDGE || c.inb[k]) {
                s1 += fabs(ux[k]) + fabs(ut[k]);
                s2 = fma(ux[k], ux[k], fma(ut[k], ut[k], s2));
            }
        }
        l1 += double(s1);
        l2 += double(s2);
    }
    __device__ __forceinline__ void sum_res(int m, const T (&a)[V])
    {
        if (!(own(m) && c.lane_out)) return;
#pragma unroll
        for (int k = 0; k < V; ++k) {
            if (EDGE && !c.inb[k]) continue;
            const double av = double(a[k]);
            aa = fma(av, av, aa);
        }
    }

    // step on row i; S = (i - ibeg) mod 4; TWO: two iterations (else one)
    template <int S, bool TWO>
    __device__ __forceinline__ void step(int i)
    {
        constexpr int C = S, PV = (S + 3) & 3, PV2 = (S + 2) & 3, NX = (S + 1) & 3;
        constexpr int P = S & 1, Q = P ^ 1;
        load(i + 1, LX[NX], LT[NX], LP[NX], LS[NX]);
        // P1 of row i
        prox_row(LX[C], LT[C], LP[C], LP[PV], i > 0, P1X[P], P1T[P]);
        // A_k and A_{k+1} of row i - 1, then D1
        const int m = i - 1;
        const bool nxt = i < c.nr, prv = m > 0;
        T a0[V], a1[V];
        div_row<T, EDGE>(c, nxt, prv, LX[PV], LX[C], LT[PV], lane_next(LT[PV][0]), LS[PV], a0);
        div_row<T, EDGE>(c, nxt, prv, P1X[Q], P1X[P], P1T[Q], lane_next(P1T[Q][0]), LS[PV], a1);
        dual_row(a1, a0, LP[PV], D1[Q]);
        if constexpr (!TWO) {
            // one iteration: u_{k+1} of row i - 1 and phi_{k+1} of row i - 1 are the outputs
            store(c.uxo, store_off(m), P1X[Q]);
            store(c.uto, store_off(m), P1T[Q]);
            store(c.phio, store_off(m), D1[Q]);
            sum_flux(m, P1X[Q], P1T[Q]);
            sum_res(m, a1);
#pragma unroll
            for (int k = 0; k < V; ++k) A1[Q][k] = a1[k];
        } else {
#pragma unroll
            for (int k = 0; k < V; ++k) A1[Q][k] = a1[k];
            // P2 of row i - 1 (phi_{k+1} of rows i - 1 and i - 2)
            prox_row(P1X[Q], P1T[Q], D1[Q], D1[P], m > 0, P2X[Q], P2T[Q]);
            store(c.uxo, store_off(m), P2X[Q]);
            store(c.uto, store_off(m), P2T[Q]);
            sum_flux(m, P2X[Q], P2T[Q]);
            // A_{k+2} and D2 of row i - 2
            const int m2 = i - 2;
            T a2[V], d2[V];
            div_row<T, EDGE>(c, i - 1 < c.nr, m2 > 0, P2X[P], P2X[Q], P2T[P], lane_next(P2T[P][0]),
                             LS[PV2], a2);
            dual_row(a2, A1[P], D1[P], d2);
            store(c.phio, store_off(m2), d2);
            sum_res(m2, a2);
        }
    }

    template <bool TWO>
    __device__ __forceinline__ void run()
    {
        load(c.ibeg, LX[0], LT[0], LP[0], LS[0]);
        int i = c.ibeg;
        for (; i + 3 <= iend; i += 4) {
            step<0, TWO>(i);
            step<1, TWO>(i + 1);
            step<2, TWO>(i + 2);
            step<3, TWO>(i + 3);
        }
        if (i <= iend) {
            step<0, TWO>(i++);
            if (i <= iend) {
                step<1, TWO>(i++);
                if (i <= iend) step<2, TWO>(i++);
            }
        }
    }
};

// The upward march of the two-iteration sweep, used on odd strips so that the two
// tiles at every strip boundary read their shared rows (two either side) at about the
// same time, as in PipeUp.  Row r's primal update needs phi of row r - 1 (the
// backward x-difference) and its residual the flux of row r + 1 (the forward
// difference), so marching up from the last loaded row each stage runs one row
// behind the one before it: at step i (row i just loaded) the wave forms P1 of row
// i + 1, A_k, A_{k+1} and D1 of row i + 1, then P2, A_{k+2} and D2 of row i + 2.
// Every row is computed by the same calls on the same operands as in Pipe2, so the
// fields are bitwise the same; only the order in which the stop rule's sums add the
// rows differs.  Register sets: loaded rows by (ilast - row) mod 4, computed rows by
// parity of that, as in Pipe2.  Rows above the grid (i < 0) are virtual: nothing is
// loaded for them and their weights in the operators are zero.
template <typename T, bool EDGE>
struct Pipe2Up : Pipe2<T, EDGE> {
    using B = Pipe2<T, EDGE>;
    using B::c;
    using B::LX;
    using B::LT;
    using B::LP;
    using B::LS;
    using B::P1X;
    using B::P1T;
    using B::A1;
    using B::D1;
    using B::P2X;
    using B::P2T;
    static constexpr int V = Vec<T>::N;

    __device__ explicit Pipe2Up(const TileCtx<T>& ctx) : B(ctx) {}

    // rows outside [ibeg, ilast] go out of range instead of to memory
    __device__ __forceinline__ void load_row(int i, T (&ux)[V], T (&ut)[V], T (&ph)[V], T (&sv)[V])
    {
        const uint32_t o = (i >= c.ibeg && i <= c.ilast) ? c.vb_ld + (uint32_t)i * c.row_bytes : OOB;
        bload(c.uxi, o, ux);
        bload(c.uti, o, ut);
        bload(c.phi_i, o, ph);
        bload(c.si, o, sv);
    }

    // step on row i; S = (ilast - i) mod 4; TWO: two iterations (else one)
    template <int S, bool TWO>
    __device__ __forceinline__ void step(int i)
    {
        constexpr int C = S, U1 = (S + 3) & 3, U2 = (S + 2) & 3, NX = (S + 1) & 3;
        constexpr int P = S & 1, Q = P ^ 1;  // computed rows: i + 1 in set Q, i + 2 in set P
        load_row(i - 1, LX[NX], LT[NX], LP[NX], LS[NX]);
        // P1 of row i + 1 (phi_k of rows i + 1 and i)
        const int m = i + 1;
        this->prox_row(LX[U1], LT[U1], LP[U1], LP[C], m > 0, P1X[Q], P1T[Q]);
        // A_k and A_{k+1} of row i + 1 (fluxes of rows i + 1 and i + 2), then D1
        const bool nxt = m + 1 < c.nr, prv = m > 0;
        T a0[V], a1[V];
        div_row<T, EDGE>(c, nxt, prv, LX[U1], LX[U2], LT[U1], lane_next(LT[U1][0]), LS[U1], a0);
        div_row<T, EDGE>(c, nxt, prv, P1X[Q], P1X[P], P1T[Q], lane_next(P1T[Q][0]), LS[U1], a1);
        this->dual_row(a1, a0, LP[U1], D1[Q]);
#pragma unroll
        for (int k = 0; k < V; ++k) A1[Q][k] = a1[k];
        if constexpr (!TWO) {
            this->store(c.uxo, this->store_off(m), P1X[Q]);
            this->store(c.uto, this->store_off(m), P1T[Q]);
            this->store(c.phio, this->store_off(m), D1[Q]);
            this->sum_flux(m, P1X[Q], P1T[Q]);
            this->sum_res(m, a1);
        } else {
            // P2 of row i + 2 (phi_{k+1} of rows i + 2 and i + 1)
            const int m2 = i + 2;
            this->prox_row(P1X[P], P1T[P], D1[P], D1[Q], m2 > 0, P2X[P], P2T[P]);
            this->store(c.uxo, this->store_off(m2), P2X[P]);
            this->store(c.uto, this->store_off(m2), P2T[P]);
            this->sum_flux(m2, P2X[P], P2T[P]);
            // A_{k+2} of row i + 2 (P2 of rows i + 2 and i + 3) and D2
            T a2[V], d2[V];
            div_row<T, EDGE>(c, m2 + 1 < c.nr, m2 > 0, P2X[P], P2X[Q], P2T[P], lane_next(P2T[P][0]),
                             LS[U2], a2);
            this->dual_row(a2, A1[P], D1[P], d2);
            this->store(c.phio, this->store_off(m2), d2);
            this->sum_res(m2, a2);
        }
    }

    // steps from the last loaded row up to (and including) row iend_up
    template <bool TWO>
    __device__ __forceinline__ void run_up(int iend_up)
    {
        load_row(c.ilast, LX[0], LT[0], LP[0], LS[0]);
        int i = c.ilast;
        for (; i - 3 >= iend_up; i -= 4) {
            step<0, TWO>(i);
            step<1, TWO>(i - 1);
            step<2, TWO>(i - 2);
            step<3, TWO>(i - 3);
        }
        if (i >= iend_up) {
            step<0, TWO>(i--);
            if (i >= iend_up) {
                step<1, TWO>(i--);
                if (i >= iend_up) step<2, TWO>(i--);
            }
        }
    }
};

// The view of one tile for a fixed-step sweep of up to K iterations: the strip's rows
// with K halo rows above and below it, the lane's samples, and the buffer descriptors
// of the fields it reads (buffer parity pb) and writes.  The steps are set once the
// gather's decision is taken (set_steps).
template <typename T>
__device__ __forceinline__ TileCtx<T> fixed_tile_ctx(const SweepArgs<T>& a, const Tile& tl, const GatherMeta& gm,
                                                     int pb, int K)
{
    constexpr int V = Vec<T>::N;
    const int lane = threadIdx.x & (WAVE - 1);
    const int qb = pb ^ 1;
    TileCtx<T> c;
    c.nr = gm.nr;
    c.ld = gm.ld;
    const int nt = gm.nt;
    c.r0 = tl.r0;
    c.rend = min(tl.r0 + gm.rows, gm.nr);
    c.ibeg = max(tl.r0 - K, 0);
    c.ilast = min(c.rend + K - 1, gm.nr - 1);
    const int j0 = tl.c0 - V + V * lane;
    const bool lane_load = (lane <= HALO_LANE_R) && (j0 >= 0) && (j0 < nt);
    c.lane_out = (lane >= 1) && (lane <= OUT_LANES) && lane_load;
#pragma unroll
    for (int k = 0; k < V; ++k) {
        const int j = j0 + k;
        c.inb[k] = (j >= 0) && (j < nt);
        c.jgt0[k] = j > 0;
        c.jlt[k] = j + 1 < nt;
    }
    c.idx = T(1.0 / gm.dx);
    c.idt = T(1.0 / gm.dt);
    c.row_bytes = (uint32_t)(gm.ld * sizeof(T));
    c.vb_ld = lane_load ? (uint32_t)(j0 * (int)sizeof(T)) : OOB;
    c.vb_st = c.lane_out ? (uint32_t)(j0 * (int)sizeof(T)) : OOB;
    const int bytes = (int)((int64_t)gm.nr * gm.ld * sizeof(T));
    auto rs = [&](const T* f) {
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(f + gm.poff), 0, bytes, 0x00020000);
    };
    c.uxi = rs(a.ux[pb]);
    c.uti = rs(a.ut[pb]);
    c.phi_i = rs(a.phi[pb]);
    c.si = rs(a.s);
    c.uxo = rs(a.ux[qb]);
    c.uto = rs(a.ut[qb]);
    c.phio = rs(a.phi[qb]);
    c.ri = c.si;
    c.ro = c.phio;
    return c;
}

template <typename T>
__device__ __forceinline__ void set_steps(TileCtx<T>& c, const SweepArgs<T>& a, const Decision2& d)
{
    c.beta = T(d.beta);
    c.theta = T(1.0);
    c.alpha = T(d.alpha);
    c.inv = T(1.0 / (1.0 + a.sc.eps * d.alpha));
}

// A gather's stop-rule sums of this tile, written to its partial-sum slot.
template <typename T>
__device__ __forceinline__ void write_fixed_sums(const SweepArgs<T>& a, const Tile& tl, int q, double aa, double l1,
                                                 double l2)
{
    double r[NPART];
#pragma unroll
    for (int m = 0; m < NPART; ++m) r[m] = 0.0;
    r[0] = wave_sum(aa);
    r[6] = wave_sum(l1);
    r[7] = wave_sum(l2);
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        double* __restrict__ dst = a.part[q] + (int64_t)tl.slot * NPART;
#pragma unroll
        for (int m = 0; m < NPART; ++m) dst[m] = r[m];
    }
}

template <typename T, bool EDGE>
__device__ void sweep_tile2(const SweepArgs<T>& a, const Tile& tl, const GatherMeta& gm, int p, int pb, int w,
                            double* red, bool up)
{
    TileCtx<T> c = fixed_tile_ctx<T>(a, tl, gm, pb, 2);
    const Decision2 d = decide_fixedk<T, 2>(a, p, tl.g, gm, tl.slot == gm.tile_base, pb, w, red);
    if (d.steps == 0) return;
    set_steps<T>(c, a, d);
    // one pipeline object for both directions: with the direction a run-time (wave-
    // uniform) branch the kernel keeps the register count of one direction (118
    // VGPRs in FP32, four waves per SIMD) where two instantiations took 140
    Pipe2Up<T, EDGE> P(c);
    if (up) {
        // the first own row's outputs come from the step one (P1, D1) or two (P2, D2)
        // rows above it
        if (d.steps == 2) P.template run_up<true>(c.r0 - 2);
        else P.template run_up<false>(c.r0 - 1);
    } else {
        // the last own row's D_K comes from the step K - 1 rows below it (rows past
        // the grid are virtual: nothing is loaded there and their weights are zero)
        P.iend = c.rend + d.steps - 1;
        if (d.steps == 2) P.template run<true>();
        else P.template run<false>();
    }
    write_fixed_sums<T>(a, tl, p ^ 1, P.aa, P.l1, P.l2);
}


// ======================================================================================
// Plain PDHG with fixed steps, three iterations per HBM pass (iters_per_sweep = 3): the
// two-iteration pipeline with a third stage.  Stage s (1, 2, 3) forms, at step i, the
// primal update P_s of row i - s + 1 and the residuals A_{k+s-1}, A_{k+s} and dual
// update D_s of row i - s, each from the stage before it one step earlier:
//   P1 of row i; A_k, A_{k+1}, D1 of row i - 1;
//   P2 of row i - 1; A_{k+2}, D2 of row i - 2;
//   P3 of row i - 2; A_{k+3}, D3 of row i - 3,
// with the calls and operands of the one-iteration sweep, so the fields are bitwise
// its fields.  A tile loads three rows above and three below its own rows (its halo
// lanes' four FP32 samples cover the three samples either way; FP64 lanes hold two,
// so the plan rejects three iterations per sweep in FP64).  u^x, u^t, phi of loaded
// rows sit in sets by row mod 4 (rows i - 1, i, and i + 1 in flight); s is needed
// three rows back, so row i + 1's s is loaded at the end of step i, into the set of
// row i - 3 that stage 3 has just read, and first used two steps later.  A sweep of
// one or two iterations (to realign a count, or at max_iter) runs the first stages
// only, with the one- or two-row halo.  Even strips march down, odd strips up
// (Pipe3Up).  The same 28 bytes per cell as the two-iteration sweep now carry three
// iterations (9.3 per iteration).
// ======================================================================================

template <typename T, bool EDGE>
struct Pipe3 : Pipe2<T, EDGE> {
    using B = Pipe2<T, EDGE>;
    using B::c;
    using B::LX;
    using B::LT;
    using B::LP;
    using B::LS;
    using B::P1X;
    using B::P1T;
    using B::A1;
    using B::D1;
    using B::P2X;
    using B::P2T;
    static constexpr int V = Vec<T>::N;
    T A2[2][V], D2[2][V];    // A_{k+2}, phi_{k+2}: rows i - 2 and i - 3
    T P3X[2][V], P3T[2][V];  // u_{k+3}: rows i - 2 and i - 3

    __device__ explicit Pipe3(const TileCtx<T>& ctx) : B(ctx)
    {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            zero(A2[b]); zero(D2[b]); zero(P3X[b]); zero(P3T[b]);
        }
    }

    // rows outside [ibeg, ilast] go out of range instead of to memory
    __device__ __forceinline__ uint32_t roff(int i) const
    {
        return (i >= c.ibeg && i <= c.ilast) ? c.vb_ld + (uint32_t)i * c.row_bytes : OOB;
    }
    __device__ __forceinline__ void load_f(int i, T (&ux)[V], T (&ut)[V], T (&ph)[V])
    {
        const uint32_t o = roff(i);
        bload(c.uxi, o, ux);
        bload(c.uti, o, ut);
        bload(c.phi_i, o, ph);
    }
    __device__ __forceinline__ void load_s(int i, T (&sv)[V]) { bload(c.si, roff(i), sv); }

    // step on row i; S = (i - ibeg) mod 4; K: iterations this sweep runs (1, 2 or 3)
    template <int S, int K>
    __device__ __forceinline__ void step(int i)
    {
        constexpr int C = S, PV = (S + 3) & 3, NX = (S + 1) & 3;
        constexpr int M1 = PV, M2 = (S + 2) & 3, M3 = (S + 1) & 3;  // s of rows i - 1, i - 2, i - 3
        constexpr int P = S & 1, Q = P ^ 1;
        load_f(i + 1, LX[NX], LT[NX], LP[NX]);
        // stage 1: P1 of row i, then A_k, A_{k+1} and D1 of row i - 1
        this->prox_row(LX[C], LT[C], LP[C], LP[PV], i > 0, P1X[P], P1T[P]);
        const int m = i - 1;
        const bool nxt = i < c.nr, prv = m > 0;
        T a0[V], a1[V];
        div_row<T, EDGE>(c, nxt, prv, LX[PV], LX[C], LT[PV], lane_next(LT[PV][0]), LS[M1], a0);
        div_row<T, EDGE>(c, nxt, prv, P1X[Q], P1X[P], P1T[Q], lane_next(P1T[Q][0]), LS[M1], a1);
        this->dual_row(a1, a0, LP[PV], D1[Q]);
#pragma unroll
        for (int k = 0; k < V; ++k) A1[Q][k] = a1[k];
        if constexpr (K == 1) {
            this->store(c.uxo, this->store_off(m), P1X[Q]);
            this->store(c.uto, this->store_off(m), P1T[Q]);
            this->store(c.phio, this->store_off(m), D1[Q]);
            this->sum_flux(m, P1X[Q], P1T[Q]);
            this->sum_res(m, a1);
        } else {
            // stage 2: P2 of row i - 1, then A_{k+2} and D2 of row i - 2
            this->prox_row(P1X[Q], P1T[Q], D1[Q], D1[P], m > 0, P2X[Q], P2T[Q]);
            const int m2 = i - 2;
            T a2[V];
            div_row<T, EDGE>(c, m < c.nr, m2 > 0, P2X[P], P2X[Q], P2T[P], lane_next(P2T[P][0]), LS[M2], a2);
            if constexpr (K == 2) {
                this->store(c.uxo, this->store_off(m), P2X[Q]);
                this->store(c.uto, this->store_off(m), P2T[Q]);
                this->sum_flux(m, P2X[Q], P2T[Q]);
                T d2[V];
                this->dual_row(a2, A1[P], D1[P], d2);
                this->store(c.phio, this->store_off(m2), d2);
                this->sum_res(m2, a2);
            } else {
                this->dual_row(a2, A1[P], D1[P], D2[P]);
#pragma unroll
                for (int k = 0; k < V; ++k) A2[P][k] = a2[k];
                // stage 3: P3 of row i - 2, then A_{k+3} and D3 of row i - 3
                this->prox_row(P2X[P], P2T[P], D2[P], D2[Q], m2 > 0, P3X[P], P3T[P]);
                this->store(c.uxo, this->store_off(m2), P3X[P]);
                this->store(c.uto, this->store_off(m2), P3T[P]);
                this->sum_flux(m2, P3X[P], P3T[P]);
                const int m3 = i - 3;
                T a3[V], d3[V];
                div_row<T, EDGE>(c, m2 < c.nr, m3 > 0, P3X[Q], P3X[P], P3T[Q], lane_next(P3T[Q][0]),
                                 LS[M3], a3);
                this->dual_row(a3, A2[Q], D2[Q], d3);
                this->store(c.phio, this->store_off(m3), d3);
                this->sum_res(m3, a3);
            }
        }
        // s of row i + 1, into the set stage 3 read above (first used at step i + 2)
        load_s(i + 1, LS[NX]);
    }

    template <int K>
    __device__ __forceinline__ void run()
    {
        load_f(c.ibeg, LX[0], LT[0], LP[0]);
        load_s(c.ibeg, LS[0]);
        const int iend = this->iend;
        int i = c.ibeg;
        for (; i + 3 <= iend; i += 4) {
            step<0, K>(i);
            step<1, K>(i + 1);
            step<2, K>(i + 2);
            step<3, K>(i + 3);
        }
        if (i <= iend) {
            step<0, K>(i++);
            if (i <= iend) {
                step<1, K>(i++);
                if (i <= iend) step<2, K>(i++);
            }
        }
    }
};

// The upward march of the three-iteration sweep, on odd strips (as Pipe2Up for two
// iterations): marching up, stage s forms at step i the primal update P_s of row
// i + s (it needs the dual iterate of the row above, row i + s - 1) and A_{k+s}, D_s
// of row i + s (the divergence needs the flux of row i + s + 1, formed one step
// earlier).  Same calls on the same operands as the downward march, so the fields are
// bitwise the same.  Loaded u^x, u^t, phi by (ilast - row) mod 4; s of row i - 1 is
// loaded at the end of step i into the set of row i + 3, which stage 3 has just read.
template <typename T, bool EDGE>
struct Pipe3Up : Pipe3<T, EDGE> {
    using B3 = Pipe3<T, EDGE>;
    using B3::c;
    using B3::LX;
    using B3::LT;
    using B3::LP;
    using B3::LS;
    using B3::P1X;
    using B3::P1T;
    using B3::A1;
    using B3::D1;
    using B3::P2X;
    using B3::P2T;
    using B3::A2;
    using B3::D2;
    using B3::P3X;
    using B3::P3T;
    static constexpr int V = Vec<T>::N;

    __device__ explicit Pipe3Up(const TileCtx<T>& ctx) : B3(ctx) {}

    // step on row i; S = (ilast - i) mod 4; K: iterations this sweep runs
    template <int S, int K>
    __device__ __forceinline__ void step_up(int i)
    {
        constexpr int C = S, U1 = (S + 3) & 3, U2 = (S + 2) & 3, U3 = (S + 1) & 3, NX = (S + 1) & 3;
        constexpr int P = S & 1, Q = P ^ 1;  // computed rows: i + 1, i + 3 in set Q; i + 2, i + 4 in P
        this->load_f(i - 1, LX[NX], LT[NX], LP[NX]);
        // stage 1: P1, A_k, A_{k+1} and D1 of row i + 1
        const int m = i + 1;
        this->prox_row(LX[U1], LT[U1], LP[U1], LP[C], m > 0, P1X[Q], P1T[Q]);
        const bool nxt = m + 1 < c.nr, prv = m > 0;
        T a0[V], a1[V];
        div_row<T, EDGE>(c, nxt, prv, LX[U1], LX[U2], LT[U1], lane_next(LT[U1][0]), LS[U1], a0);
        div_row<T, EDGE>(c, nxt, prv, P1X[Q], P1X[P], P1T[Q], lane_next(P1T[Q][0]), LS[U1], a1);
        this->dual_row(a1, a0, LP[U1], D1[Q]);
#pragma unroll
        for (int k = 0; k < V; ++k) A1[Q][k] = a1[k];
        if constexpr (K == 1) {
            this->store(c.uxo, this->store_off(m), P1X[Q]);
            this->store(c.uto, this->store_off(m), P1T[Q]);
            this->store(c.phio, this->store_off(m), D1[Q]);
            this->sum_flux(m, P1X[Q], P1T[Q]);
            this->sum_res(m, a1);
        } else {
            // stage 2: P2, A_{k+2} and D2 of row i + 2
            const int m2 = i + 2;
            this->prox_row(P1X[P], P1T[P], D1[P], D1[Q], m2 > 0, P2X[P], P2T[P]);
            T a2[V];
            div_row<T, EDGE>(c, m2 + 1 < c.nr, m2 > 0, P2X[P], P2X[Q], P2T[P], lane_next(P2T[P][0]),
                             LS[U2], a2);
            if constexpr (K == 2) {
                this->store(c.uxo, this->store_off(m2), P2X[P]);
                this->store(c.uto, this->store_off(m2), P2T[P]);
                this->sum_flux(m2, P2X[P], P2T[P]);
                T d2[V];
                this->dual_row(a2, A1[P], D1[P], d2);
                this->store(c.phio, this->store_off(m2), d2);
                this->sum_res(m2, a2);
            } else {
                this->dual_row(a2, A1[P], D1[P], D2[P]);
#pragma unroll
                for (int k = 0; k < V; ++k) A2[P][k] = a2[k];
                // stage 3: P3, A_{k+3} and D3 of row i + 3
                const int m3 = i + 3;
                this->prox_row(P2X[Q], P2T[Q], D2[Q], D2[P], m3 > 0, P3X[Q], P3T[Q]);
                this->store(c.uxo, this->store_off(m3), P3X[Q]);
                this->store(c.uto, this->store_off(m3), P3T[Q]);
                this->sum_flux(m3, P3X[Q], P3T[Q]);
                T a3[V], d3[V];
                div_row<T, EDGE>(c, m3 + 1 < c.nr, m3 > 0, P3X[Q], P3X[P], P3T[Q], lane_next(P3T[Q][0]),
                                 LS[U3], a3);
                this->dual_row(a3, A2[Q], D2[Q], d3);
                this->store(c.phio, this->store_off(m3), d3);
                this->sum_res(m3, a3);
            }
        }
        // s of row i - 1, into the set stage 3 read above (first used at step i - 2)
        this->load_s(i - 1, LS[NX]);
    }

    // steps from the last loaded row up to (and including) row iend_up
    template <int K>
    __device__ __forceinline__ void run_up(int iend_up)
    {
        this->load_f(c.ilast, LX[0], LT[0], LP[0]);
        this->load_s(c.ilast, LS[0]);
        int i = c.ilast;
        for (; i - 3 >= iend_up; i -= 4) {
            step_up<0, K>(i);
            step_up<1, K>(i - 1);
            step_up<2, K>(i - 2);
            step_up<3, K>(i - 3);
        }
        if (i >= iend_up) {
            step_up<0, K>(i--);
            if (i >= iend_up) {
                step_up<1, K>(i--);
                if (i >= iend_up) step_up<2, K>(i--);
            }
        }
    }
};

template <typename T, bool EDGE>
__device__ void sweep_tile3(const SweepArgs<T>& a, const Tile& tl, const GatherMeta& gm, int p, int pb, int w,
                            double* red, bool up)
{
    TileCtx<T> c = fixed_tile_ctx<T>(a, tl, gm, pb, 3);
    const Decision2 d = decide_fixedk<T, 3>(a, p, tl.g, gm, tl.slot == gm.tile_base, pb, w, red);
    if (d.steps == 0) return;
    set_steps<T>(c, a, d);
    // one pipeline object for both directions (a run-time, wave-uniform branch, as in
    // the two-iteration sweep)
    Pipe3Up<T, EDGE> P(c);
    if (up) {
        // the first own row's outputs come from the step K rows above it
        if (d.steps == 3) P.template run_up<3>(c.r0 - 3);
        else if (d.steps == 2) P.template run_up<2>(c.r0 - 2);
        else P.template run_up<1>(c.r0 - 1);
    } else {
        // the last own row's D_K comes from the step K - 1 rows below it (rows past
        // the grid are virtual: nothing is loaded there and their weights are zero)
        P.iend = c.rend + d.steps - 1;
        if (d.steps == 3) P.template run<3>();
        else if (d.steps == 2) P.template run<2>();
        else P.template run<1>();
    }
    write_fixed_sums<T>(a, tl, p ^ 1, P.aa, P.l1, P.l2);
}

// The fixed-step sweep of K (2 or 3) iterations per launch over one tile table.  The
// four waves of a block on one running gather share its decision sums (as in k_sweep;
// every wave of such a block reaches the one barrier).  red: the block's exchange
// buffer (LDS, 4 * NPART doubles).
template <typename T, int K>
__device__ __forceinline__ void fixed_sweep(const SweepArgs<T>& a, int parity, double* red)
{
    constexpr int V = Vec<T>::N;
    constexpr int WPB = 256 / WAVE;
    const int w = uniform((int)threadIdx.x / WAVE);
    const int first = uniform(xcd_logical_block() * WPB);
    const int tid = first + w;
    if (tid >= a.ntiles) return;
    int gb = -1;
    bool split = first + WPB <= a.ntiles;
    for (int k = 0; k < WPB && split; ++k) {
        const int gk = uniform(a.tiles[first + k].g);
        if (gk < 0) continue;
        if (gb < 0) gb = gk;
        else if (gk != gb) split = false;
    }
    if (gb < 0) split = false;
    if (split) {
        const GState* sb = a.gst[parity] + gb;
        split = uniform(sb->status) == ST_RUNNING && uniform(sb->started) != 0;
    }
    const Tile tl = a.tiles[tid];
    const int g = uniform(tl.g);
    if (g < 0) {
        // padding entry: only its quarter of the block gather's decision sums
        if (split) {
            const GatherMeta mb = a.meta[gb];
            double s[NPART];
            decision_sums<NPART>(a.part[parity] + (int64_t)mb.tile_base * NPART, mb.ntiles, w, red, s);
        }
        return;
    }
    double* const xred = split ? red : nullptr;
    const GatherMeta gm = a.meta[g];
    const GState* gs = a.gst[parity] + g;
    if (gs->status != ST_RUNNING) {
        // finished gather: only carry its state to the other parity
        if (tl.slot == gm.tile_base && (threadIdx.x & (WAVE - 1)) == 0) a.gst[parity ^ 1][g] = *gs;
        return;
    }
    const int pb = parity;
    const bool edge = (tl.c0 - V < 1) || (tl.c0 + HALO_LANE_R * V > gm.nt - 1);
    // odd strips march up
    const bool up = ((tl.r0 / gm.rows) & 1) != 0;
    if constexpr (K == 2) {
        if (edge) sweep_tile2<T, true>(a, tl, gm, parity, pb, w, xred, up);
        else sweep_tile2<T, false>(a, tl, gm, parity, pb, w, xred, up);
    } else {
        if (edge) sweep_tile3<T, true>(a, tl, gm, parity, pb, w, xred, up);
        else sweep_tile3<T, false>(a, tl, gm, parity, pb, w, xred, up);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_sweep2(SweepArgs<T> a, int parity)
{
    __shared__ double red[(256 / WAVE) * NPART];
    fixed_sweep<T, 2>(a, parity, red);
}

template <typename T>
__global__ __launch_bounds__(256) void k_sweep3(SweepArgs<T> a, int parity)
{
    __shared__ double red[(256 / WAVE) * NPART];
    fixed_sweep<T, 3>(a, parity, red);
}

template <typename T>
void launch_sweep(const SweepArgs<T>& a, int parity, int grid, hipStream_t stream)
{
    if (a.ips == 3)
        hipLaunchKernelGGL((k_sweep3<T>), dim3(grid), dim3(256), 0, stream, a, parity);
    else if (a.ips == 2)
        hipLaunchKernelGGL((k_sweep2<T>), dim3(grid), dim3(256), 0, stream, a, parity);
    else if (a.l1)
        hipLaunchKernelGGL((k_sweep<T, true>), dim3(grid), dim3(256), 0, stream, a, parity);
    else
        hipLaunchKernelGGL((k_sweep<T, false>), dim3(grid), dim3(256), 0, stream, a, parity);
}

template void launch_sweep<float>(const SweepArgs<float>&, int, int, hipStream_t);
template void launch_sweep<double>(const SweepArgs<double>&, int, int, hipStream_t);

}  // namespace emd
