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
// gather does this redundantly, in a fixed order, so all agree bitwise),
// (2) applies the dual step of iteration n-1 -> n, (3) the primal update with
// alpha_n, (4) recomputes div of the new flux and the six products plus
// sum |u|, sum u^2 for the next decision.  One HBM pass per iteration: read u, phi,
// s, R (the previous residual A_n), write u, phi, R -- 36 bytes per cell in FP32.
//
// Work decomposition: a wavefront owns a tile of `rows` receiver rows by 62 * V
// time samples (V = 4 floats or 2 doubles per lane, one 16-byte vector per field).
// Lanes run along time (coalesced), the wave marches down the rows keeping the
// previous rows in registers.  The operators couple a cell to its neighbours at
// distance <= 2 rows back and 1 row ahead, and 2 samples back / 1 ahead in time:
// rows are recomputed for the halo (the march starts 2 rows early and ends 1 row
// late), and lanes 0 and 63 carry the time halo (their own samples are loaded and
// computed but never stored or reduced).
#include "emd_internal.h"
#include "emd_launch.h"

namespace emd {

struct Decision {
    double alpha;  // primal step of this sweep
    double beta;   // dual step of this sweep (0: no dual update)
    double theta;
    int run;       // 0: gather finished, nothing to do
    int prox;      // 1: compute the next primal iterate and its reductions
};

// Runs on every lane of a wave; returns the same decision on every lane.
template <typename T>
__device__ Decision decide(const SweepArgs<T>& a, int p, int g, const GatherMeta& gm,
                           bool writer)
{
    const GState* __restrict__ sin = a.gst[p] + g;
    GState* __restrict__ sout = a.gst[p ^ 1] + g;
    GState st = *sin;
    Decision d;
    d.alpha = st.alpha;
    d.beta = 0.0;
    d.theta = 0.0;
    d.run = 0;
    d.prox = 0;
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
        return d;
    }
    double q[NPART];
    reduce_records(a.part[p] + (int64_t)gm.tile_base * NPART, gm.ntiles, q);
    const double aa = q[0], ab = q[1], bb = q[2], gaa = q[3], gab = q[4], gbb = q[5];
    const double l1 = q[6], l2 = q[7];
    const SolveScalars& sc = a.sc;
    const double ak = st.alpha, tk = st.theta;
    double alpha, theta = 1.0;
    int trials = 0, status = ST_RUNNING;
    bool finite = isfinite(aa) && isfinite(ab) && isfinite(bb) && isfinite(gaa) &&
                  isfinite(gab) && isfinite(gbb) && isfinite(l1) && isfinite(l2);
    if (!finite) {
        status = ST_NONFINITE;
        alpha = ak;
    } else if (sc.ls_mode == LS_FIXED) {
        alpha = ak;
        theta = 1.0;
    } else if (sc.ls_mode == LS_REPLAY) {
        alpha = sc.replay[(int64_t)g * sc.ld_replay + st.iters];
        theta = alpha / ak;
    } else {
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
    const int p1 = p ^ 1;
    if (status == ST_RUNNING) {
        // accept iteration st.iters + 1: phi_n is written by this sweep, u_n is the
        // flux this sweep reads
        st.iters += 1;
        st.rel_res = sqrt(aa) / st.snorm;
        st.emd = gm.cm * (l1 + 0.5 * sc.eps * l2);
        st.transport = gm.cm * l1;
        st.alpha = alpha;
        st.theta = theta;
        if (st.iters % sc.check_every == 0 && st.rel_res <= sc.tol_res) status = ST_CONVERGED;
        else if (st.iters >= sc.max_iter) status = ST_MAX_ITER;
        d.run = 1;
        d.prox = (status == ST_RUNNING);
        d.alpha = alpha;
        d.beta = sc.delta * alpha;
        d.theta = theta;
        st.ubuf = p;
        st.phibuf = p1;
    } else {
        // the trial step is rejected: return the last accepted iterate (u_{n-1} is
        // still in the buffer this sweep would have written, phi_{n-1} in its input)
        st.ubuf = p1;
        st.phibuf = p;
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

template <typename T, bool PROX>
__device__ void sweep_tile(const SweepArgs<T>& a, const Tile& tl, int tid, const GatherMeta& gm,
                           const Decision& d, int p)
{
    constexpr int V = Vec<T>::N;
    const int lane = threadIdx.x & (WAVE - 1);
    const int q = p ^ 1;
    const int nr = gm.nr, nt = gm.nt, ld = gm.ld;
    const T idx = T(1.0 / gm.dx), idt = T(1.0 / gm.dt);
    const int r0 = tl.r0, c0 = tl.c0;
    const int rend = min(r0 + a.rows, nr);
    const int ibeg = max(r0 - 2, 0);
    const int ilast = min(r0 + a.rows, nr);  // == nr: a virtual row closes the last strip
    const int j0 = c0 - V + V * lane;
    const bool lane_load = (j0 >= 0) && (j0 < nt);
    const bool lane_out = (lane >= 1) && (lane <= OUT_LANES) && lane_load;
    bool inb[V], jgt0[V], jlt[V];
#pragma unroll
    for (int k = 0; k < V; ++k) {
        const int j = j0 + k;
        inb[k] = (j >= 0) && (j < nt);
        jgt0[k] = j > 0;
        jlt[k] = j + 1 < nt;
    }
    const T beta = T(d.beta), theta = T(d.theta), alpha = T(d.alpha);
    const T inv = T(1.0 / (1.0 + a.sc.eps * d.alpha));

    const int64_t base = gm.poff + j0;
    const T* __restrict__ uxi = a.ux[p] + base;
    const T* __restrict__ uti = a.ut[p] + base;
    const T* __restrict__ phi_i = a.phi[p] + base;
    const T* __restrict__ ri = a.R[p] + base;
    const T* __restrict__ si = a.s + base;
    T* __restrict__ uxo = a.ux[q] + base;
    T* __restrict__ uto = a.ut[q] + base;
    T* __restrict__ phio = a.phi[q] + base;
    T* __restrict__ ro = a.R[q] + base;

    T uxc[V], utc[V];
    if (lane_load) {
        vload(uxi + (int64_t)ibeg * ld, uxc);
        vload(uti + (int64_t)ibeg * ld, utc);
    } else {
#pragma unroll
        for (int k = 0; k < V; ++k) uxc[k] = utc[k] = T(0);
    }
    T phn_p[V], u1x_p[V], u1t_p[V], A_p[V], s_p[V], A1_pp[V], B1_pp[V];
#pragma unroll
    for (int k = 0; k < V; ++k)
        phn_p[k] = u1x_p[k] = u1t_p[k] = A_p[k] = s_p[k] = A1_pp[k] = B1_pp[k] = T(0);
    double acc[NPART];
#pragma unroll
    for (int m = 0; m < NPART; ++m) acc[m] = 0.0;

    for (int i = ibeg; i <= ilast; ++i) {
        const bool real = i < nr;
        const int64_t ro_i = (int64_t)i * ld;
        T uxn[V], utn[V], ph[V], sv[V], rv[V];
        if (i + 1 < nr && lane_load) {
            vload(uxi + ro_i + ld, uxn);
            vload(uti + ro_i + ld, utn);
        } else {
#pragma unroll
            for (int k = 0; k < V; ++k) uxn[k] = utn[k] = T(0);
        }
        if (real && lane_load) {
            vload(phi_i + ro_i, ph);
            vload(si + ro_i, sv);
            vload(ri + ro_i, rv);
        } else {
#pragma unroll
            for (int k = 0; k < V; ++k) ph[k] = sv[k] = rv[k] = T(0);
        }
        const bool own_row = (i >= r0) && (i < rend);
        T phn[V], A[V], u1x[V], u1t[V];
        if (real) {
            // (1) residual of the current flux: A = div u_n + s
            const T ut_next = __shfl_down(utc[0], 1, WAVE);
#pragma unroll
            for (int k = 0; k < V; ++k) {
                const T fx = (i + 1 < nr) ? uxn[k] : T(0);
                const T bx = (i > 0) ? uxc[k] : T(0);
                const T ftv = (k + 1 < V) ? utc[(k + 1) % V] : ut_next;
                const T ft = jlt[k] ? ftv : T(0);
                const T bt = jgt0[k] ? utc[k] : T(0);
                A[k] = (fx - bx) * idx + (ft - bt) * idt + sv[k];
            }
            // (2) dual step: phi_n = phi_{n-1} + beta (A + theta (A - R))
#pragma unroll
            for (int k = 0; k < V; ++k) phn[k] = ph[k] + beta * (A[k] + theta * (A[k] - rv[k]));
            if (own_row && lane_out) {
                T w[V];
#pragma unroll
                for (int k = 0; k < V; ++k) w[k] = inb[k] ? phn[k] : T(0);
                vstore(phio + ro_i, w);
                if constexpr (PROX) {
#pragma unroll
                    for (int k = 0; k < V; ++k) w[k] = inb[k] ? A[k] : T(0);
                    vstore(ro + ro_i, w);
                }
            }
            if constexpr (PROX) {
                // (3) primal update with the backward-difference gradient of phi_n
                const T ph_prev = __shfl_up(phn[V - 1], 1, WAVE);
                T l1 = T(0), l2 = T(0);
#pragma unroll
                for (int k = 0; k < V; ++k) {
                    const T gx = (i > 0) ? (phn[k] - phn_p[k]) * idx : T(0);
                    const T pprev = (k > 0) ? phn[(k + V - 1) % V] : ph_prev;
                    const T gt = jgt0[k] ? (phn[k] - pprev) * idt : T(0);
                    u1x[k] = shrink_scaled(uxc[k] + alpha * gx, alpha, inv);
                    u1t[k] = shrink_scaled(utc[k] + alpha * gt, alpha, inv);
                    if (inb[k]) {
                        l1 += fabs(u1x[k]) + fabs(u1t[k]);
                        l2 += u1x[k] * u1x[k] + u1t[k] * u1t[k];
                    }
                }
                if (own_row && lane_out) {
                    T w[V];
#pragma unroll
                    for (int k = 0; k < V; ++k) w[k] = inb[k] ? u1x[k] : T(0);
                    vstore(uxo + ro_i, w);
#pragma unroll
                    for (int k = 0; k < V; ++k) w[k] = inb[k] ? u1t[k] : T(0);
                    vstore(uto + ro_i, w);
                    acc[6] += double(l1);
                    acc[7] += double(l2);
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < V; ++k) phn[k] = A[k] = u1x[k] = u1t[k] = T(0);
        }

        if constexpr (PROX) {
            if (i > ibeg) {
                // (4) residual of the new flux on row i-1 and its gradient
                const int im = i - 1;
                const T u1t_next = __shfl_down(u1t_p[0], 1, WAVE);
                T A1[V], B1[V];
#pragma unroll
                for (int k = 0; k < V; ++k) {
                    const T fx = real ? u1x[k] : T(0);
                    const T bx = (im > 0) ? u1x_p[k] : T(0);
                    const T ftv = (k + 1 < V) ? u1t_p[(k + 1) % V] : u1t_next;
                    const T ft = jlt[k] ? ftv : T(0);
                    const T bt = jgt0[k] ? u1t_p[k] : T(0);
                    A1[k] = (fx - bx) * idx + (ft - bt) * idt + s_p[k];
                    B1[k] = A1[k] - A_p[k];
                }
                const T A1_prev = __shfl_up(A1[V - 1], 1, WAVE);
                const T B1_prev = __shfl_up(B1[V - 1], 1, WAVE);
                if (im >= r0 && im < rend && lane_out) {
#pragma unroll
                    for (int k = 0; k < V; ++k) {
                        const T ap = (k > 0) ? A1[(k + V - 1) % V] : A1_prev;
                        const T bp = (k > 0) ? B1[(k + V - 1) % V] : B1_prev;
                        const double gax = (im > 0) ? double((A1[k] - A1_pp[k]) * idx) : 0.0;
                        const double gbx = (im > 0) ? double((B1[k] - B1_pp[k]) * idx) : 0.0;
                        const double gat = jgt0[k] ? double((A1[k] - ap) * idt) : 0.0;
                        const double gbt = jgt0[k] ? double((B1[k] - bp) * idt) : 0.0;
                        const double av = double(A1[k]), bv = double(B1[k]);
                        if (inb[k]) {
                            acc[0] += av * av;
                            acc[1] += av * bv;
                            acc[2] += bv * bv;
                            acc[3] += gax * gax + gat * gat;
                            acc[4] += gax * gbx + gat * gbt;
                            acc[5] += gbx * gbx + gbt * gbt;
                        }
                    }
                }
#pragma unroll
                for (int k = 0; k < V; ++k) {
                    A1_pp[k] = A1[k];
                    B1_pp[k] = B1[k];
                }
            }
#pragma unroll
            for (int k = 0; k < V; ++k) {
                u1x_p[k] = u1x[k];
                u1t_p[k] = u1t[k];
            }
        }
#pragma unroll
        for (int k = 0; k < V; ++k) {
            phn_p[k] = phn[k];
            A_p[k] = A[k];
            s_p[k] = sv[k];
            uxc[k] = uxn[k];
            utc[k] = utn[k];
        }
    }

    if constexpr (PROX) {
#pragma unroll
        for (int m = 0; m < NPART; ++m) acc[m] = wave_sum(acc[m]);
        if (lane == 0) {
            double* __restrict__ dst = a.part[q] + (int64_t)tid * NPART;
#pragma unroll
            for (int m = 0; m < NPART; ++m) dst[m] = acc[m];
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_sweep(SweepArgs<T> a, int parity)
{
    const int tid = uniform(xcd_logical_block() * (blockDim.x / WAVE) + threadIdx.x / WAVE);
    if (tid >= a.ntiles) return;
    const Tile tl = a.tiles[tid];
    const int g = uniform(tl.g);
    const GatherMeta gm = a.meta[g];
    const Decision d = decide(a, parity, g, gm, tid == gm.tile_base);
    if (!d.run) return;
    if (d.prox) sweep_tile<T, true>(a, tl, tid, gm, d, parity);
    else sweep_tile<T, false>(a, tl, tid, gm, d, parity);
}

template <typename T>
void launch_sweep(const SweepArgs<T>& a, int parity, int grid, hipStream_t stream)
{
    hipLaunchKernelGGL(k_sweep<T>, dim3(grid), dim3(256), 0, stream, a, parity);
}

template void launch_sweep<float>(const SweepArgs<float>&, int, int, hipStream_t);
template void launch_sweep<double>(const SweepArgs<double>&, int, int, hipStream_t);

}  // namespace emd
