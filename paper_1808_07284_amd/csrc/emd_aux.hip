// emd_aux.hip -- the once-per-solve passes around the PDHG sweeps: the signed-data
// recombination and normalisation (Section 2.1 of the paper), moving the caller's
// batch into the padded solver state and back, per-gather start-up and results,
// and the adjoint source (Section 2.3).
//
// All passes use the sweep tile table, one wavefront per entry, so per-gather sums
// are built from per-tile partials (one slot per tile, contiguous per gather) reduced
// in a fixed order (deterministic).  Passes between the padded state and the caller's
// layout cover the tile itself (`rows` receiver rows by 56 * V time samples, lanes
// 1..56 with V samples each); passes that touch only the caller's layout (decompose,
// adjoint, least squares) walk a contiguous chunk of the gather's elements per slot,
// consecutive lanes on consecutive elements.
#include "emd_internal.h"
#include "emd_launch.h"

namespace emd {

namespace {

struct TileView {
    int tid, slot, g, r0, rend, j0, lane;
    bool active;  // this lane owns samples in the tile
};

template <typename T>
__device__ __forceinline__ TileView tile_view(const AuxArgs<T>& a, GatherMeta& gm, bool& ok)
{
    constexpr int V = Vec<T>::N;
    TileView v;
    v.tid = uniform(xcd_logical_block() * (blockDim.x / WAVE) + threadIdx.x / WAVE);
    ok = v.tid < a.ntiles;
    if (!ok) return v;
    const Tile tl = a.tiles[v.tid];
    v.g = uniform(tl.g);
    ok = v.g >= 0;  // padding entries do nothing
    if (!ok) return v;
    v.slot = uniform(tl.slot);
    gm = a.meta[v.g];
    v.lane = threadIdx.x & (WAVE - 1);
    v.r0 = tl.r0;
    v.rend = min(tl.r0 + gm.rows, gm.nr);
    v.j0 = tl.c0 - V + V * v.lane;
    v.active = (v.lane >= 1) && (v.lane <= OUT_LANES) && (v.j0 >= 0) && (v.j0 < gm.nt);
    return v;
}

__device__ __forceinline__ void write_record(double* part, int slot, const double (&acc)[NPART])
{
    const int lane = threadIdx.x & (WAVE - 1);
    double r[NPART];
#pragma unroll
    for (int m = 0; m < NPART; ++m) r[m] = wave_sum(acc[m]);
    if (lane == 0) {
#pragma unroll
        for (int m = 0; m < NPART; ++m) part[(int64_t)slot * NPART + m] = r[m];
    }
}

// The elements whose sums go to a tile's slot, for the passes over the caller's
// layout: gather g's nr * nt elements (row-major) cut into ntiles contiguous chunks,
// chunk c for slot tile_base + c.  Offsets are relative to the gather's first element.
__device__ __forceinline__ void slot_chunk(const TileView& tv, const GatherMeta& gm, int64_t& lo, int64_t& hi)
{
    const int64_t n = (int64_t)gm.nr * gm.nt;
    const int64_t per = (n + gm.ntiles - 1) / gm.ntiles;
    lo = min((int64_t)(tv.slot - gm.tile_base) * per, n);
    hi = min(lo + per, n);
}

// A wave takes kUnroll strided elements per step (e, e + 64, ...), all loads of a
// step issued before any is used; elements at or past hi read as zero.
constexpr int kUnroll = 4;

template <typename T>
__device__ __forceinline__ void load_step(const T* __restrict__ p, int64_t e, int64_t hi, double (&x)[kUnroll])
{
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
        const int64_t k = e + (int64_t)u * WAVE;
        x[u] = k < hi ? double(p[k]) : 0.0;
    }
}

// ------------------------------------------------------------------ solve start

// s, u, phi from the caller's layout into buffer 0 of the padded state; R = 0.
// Partials: sum s^2, count of non-finite s.
template <typename T>
__global__ __launch_bounds__(256) void k_copy_in(AuxArgs<T> a, int warm)
{
    constexpr int V = Vec<T>::N;
    GatherMeta gm;
    bool ok;
    const TileView tv = tile_view(a, gm, ok);
    if (!ok) return;
    double acc[NPART];
#pragma unroll
    for (int m = 0; m < NPART; ++m) acc[m] = 0.0;
    for (int i = tv.r0; i < tv.rend; ++i) {
        if (!tv.active) continue;
        const int64_t pr = gm.poff + (int64_t)i * gm.ld + tv.j0;
        const int64_t ur = gm.uoff + (int64_t)i * gm.nt + tv.j0;
        T sv[V], ux[V], ut[V], ph[V], z[V];
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const bool in = tv.j0 + k < gm.nt;
            sv[k] = in ? a.s_user[ur + k] : T(0);
            ux[k] = (in && warm && a.u_user_in) ? a.u_user_in[ur + k] : T(0);
            ut[k] = (in && warm && a.u_user_in) ? a.u_user_in[a.batch_len + ur + k] : T(0);
            ph[k] = (in && warm && a.phi_user_in) ? a.phi_user_in[ur + k] : T(0);
            z[k] = T(0);
            if (in) {
                acc[0] += double(sv[k]) * double(sv[k]);
                acc[1] += isfinite(double(sv[k])) ? 0.0 : 1.0;
            }
        }
        vstore(a.s_pad + pr, sv);
        vstore(a.ux[0] + pr, ux);
        vstore(a.ut[0] + pr, ut);
        vstore(a.phi[0] + pr, ph);
        vstore(a.R[0] + pr, z);
    }
    write_record(a.part, tv.slot, acc);
}

// One wavefront per gather: ||s||, start status and the parity-0 scalar state.
template <typename T>
__global__ __launch_bounds__(64) void k_gather_init(AuxArgs<T> a)
{
    const int g = blockIdx.x;
    const GatherMeta gm = a.meta[g];
    double q[NPART];
    reduce_records(a.part + (int64_t)gm.tile_base * NPART, gm.ntiles, q);
    GState st;
    st.snorm = sqrt(q[0]);
    st.alpha = gm.alpha1;
    st.theta = 1.0;
    st.alpha_max = a.alpha_max_factor > 0.0 ? a.alpha_max_factor * gm.alpha1 : INFINITY;
    st.rel_res = 1.0;
    st.emd = 0.0;
    st.transport = 0.0;
    st.iters = 0;
    st.trials = 0;
    st.started = 0;
    st.ubuf = 0;
    st.phibuf = 0;
    st.flip = 0;
    st.ls_base = 0;
    int status = ST_RUNNING;
    if (q[1] != 0.0 || !isfinite(st.snorm)) {
        status = ST_NONFINITE;
        st.rel_res = NAN;
        st.emd = NAN;
        st.transport = NAN;
    } else if (a.mass_mode == MASS_NONE && a.mass != nullptr &&
               fabs(a.mass[3 * g] - a.mass[3 * g + 1]) >
                   a.mass_tol * fmax(a.mass[3 * g], a.mass[3 * g + 1])) {
        status = ST_MASS_IMBALANCE;
        st.rel_res = NAN;
        st.emd = NAN;
        st.transport = NAN;
    } else if (st.snorm == 0.0) {
        status = ST_ZERO_SOURCE;
        st.rel_res = 0.0;
    }
    if (a.resume && status == ST_RUNNING) {
        // continue from the checkpointed iteration: its steps and counts; the first
        // sweep (started == 0) redoes that iteration's primal update with alpha
        const ResumeRec r = a.resume[g];
        st.alpha = r.alpha;
        st.theta = r.theta;
        st.iters = r.iters;
        st.trials = r.trials;
        if (r.status != ST_RUNNING && r.status != ST_MAX_ITER) {
            // the gather had finished: it keeps its outcome and is never swept, so
            // the u and phi copied in above are what the solve returns for it
            status = r.status;
            st.rel_res = r.rel_res;
            st.emd = r.primal;
            st.transport = r.transport;
        }
    }
    st.status = status;
    if (threadIdx.x == 0) {
        a.gst[g] = st;
        if (status != ST_RUNNING) atomicAdd(a.done, 1);
    }
}

__global__ void k_zero_counter(int32_t* c)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) c[0] = 0;
}

// ------------------------------------------------------------------ solve end

template <typename T>
__global__ __launch_bounds__(256) void k_copy_out(AuxArgs<T> a)
{
    constexpr int V = Vec<T>::N;
    GatherMeta gm;
    bool ok;
    const TileView tv = tile_view(a, gm, ok);
    if (!ok || !tv.active) return;
    const GState st = a.gst[tv.g];
    const bool zero = (st.status == ST_ZERO_SOURCE) || (st.status == ST_MASS_IMBALANCE);
    const T* uxs = a.ux[st.ubuf];
    const T* uts = a.ut[st.ubuf];
    const T* phs = a.phi[st.phibuf];
    for (int i = tv.r0; i < tv.rend; ++i) {
        const int64_t pr = gm.poff + (int64_t)i * gm.ld + tv.j0;
        const int64_t ur = gm.uoff + (int64_t)i * gm.nt + tv.j0;
        T ux[V], ut[V], ph[V];
        vload(uxs + pr, ux);
        vload(uts + pr, ut);
        vload(phs + pr, ph);
#pragma unroll
        for (int k = 0; k < V; ++k) {
            if (tv.j0 + k >= gm.nt) break;
            if (a.phi_user_out) a.phi_user_out[ur + k] = zero ? T(0) : ph[k];
            if (a.u_user_out) {
                a.u_user_out[ur + k] = zero ? T(0) : ux[k];
                a.u_user_out[a.batch_len + ur + k] = zero ? T(0) : ut[k];
            }
        }
    }
}

struct InfoRec {
    int32_t status, iters, ls_trials, pad;
    double rel_res, emd, transport, alpha, primal;
};

// A gather whose returned flux and potential come from iterations (not a zero,
// non-finite or unbalanced source) is priced by the Lagrangian.
__device__ __forceinline__ bool iterated(int status)
{
    return status == ST_CONVERGED || status == ST_MAX_ITER || status == ST_LS_FAIL;
}

// The potential term of the Lagrangian of Section 2.2 at the pair a solve returns:
// per tile, sum phi (div u + s) over the tile's cells, with the divergence of the
// stored flux formed in FP64 (div = minus the transpose of the backward-difference
// gradient: forward differences inside, -u/dx and -u/dt on the last row and
// column).  Reads the returned buffers of the padded state (parity-0 gather state).
template <typename T>
__global__ __launch_bounds__(256) void k_lagr_sums(AuxArgs<T> a)
{
    constexpr int V = Vec<T>::N;
    GatherMeta gm;
    bool ok;
    const TileView tv = tile_view(a, gm, ok);
    if (!ok) return;
    double acc[NPART];
#pragma unroll
    for (int m = 0; m < NPART; ++m) acc[m] = 0.0;
    const GState st = a.gst[tv.g];
    if (tv.active && iterated(st.status)) {
        const T* __restrict__ ux = a.ux[st.ubuf];
        const T* __restrict__ ut = a.ut[st.ubuf];
        const T* __restrict__ ph = a.phi[st.phibuf];
        const double idx = 1.0 / gm.dx, idt = 1.0 / gm.dt;
        for (int i = tv.r0; i < tv.rend; ++i) {
            const int64_t pr = gm.poff + (int64_t)i * gm.ld + tv.j0;
            const bool below = i + 1 < gm.nr;
            T x0[V], x1[V], t0[V], p0[V], s0[V];
            vload(ux + pr, x0);
            vload(ux + (below ? pr + gm.ld : pr), x1);
            vload(ut + pr, t0);
            vload(ph + pr, p0);
            vload(a.s_pad + pr, s0);
            // u^t of the sample after the vector (inside the padded row)
            const double tnext = tv.j0 + V < gm.nt ? double(ut[pr + V]) : 0.0;
#pragma unroll
            for (int k = 0; k < V; ++k) {
                const int j = tv.j0 + k;
                if (j >= gm.nt) break;
                double d = double(s0[k]);
                if (below) d += double(x1[k]) * idx;
                if (i > 0) d -= double(x0[k]) * idx;
                if (j + 1 < gm.nt) d += (k + 1 < V ? double(t0[(k + 1) % V]) : tnext) * idt;
                if (j > 0) d -= double(t0[k]) * idt;
                acc[0] = fma(double(p0[k]), d, acc[0]);
            }
        }
    }
    write_record(a.part, tv.slot, acc);
}

// One wavefront per gather: the Lagrangian value (from the k_lagr_sums records),
// EMD values and solve records.
template <typename T>
__global__ __launch_bounds__(64) void k_finalize(AuxArgs<T> a)
{
    const int g = blockIdx.x;
    const GatherMeta gm = a.meta[g];
    const GState st = a.gst[g];
    double q[NPART];
    reduce_records(a.part + (int64_t)gm.tile_base * NPART, gm.ntiles, q);
    const double emd = iterated(st.status) ? st.emd + gm.cm * q[0] : st.emd;
    if (threadIdx.x != 0) return;
    if (a.emd_out) a.emd_out[g] = emd;
    if (a.info_out) {
        InfoRec r;
        r.status = st.status;
        r.iters = st.iters;
        r.ls_trials = st.trials;
        r.pad = 0;
        r.rel_res = st.rel_res;
        r.emd = emd;
        r.transport = st.transport;
        r.alpha = st.alpha;
        r.primal = st.emd;
        reinterpret_cast<InfoRec*>(a.info_out)[g] = r;
    }
}

// ------------------------------------------------------------------ decompose

__device__ __forceinline__ double fpart(double pc, double po) { return fmax(pc, 0.0) + fmax(-po, 0.0); }
__device__ __forceinline__ double gpart(double pc, double po) { return fmax(po, 0.0) + fmax(-pc, 0.0); }

// partials: sum f, sum g, sum (Pcal - Pobs)
template <typename T>
__global__ __launch_bounds__(256) void k_decomp_sums(AuxArgs<T> a)
{
    GatherMeta gm;
    bool ok;
    const TileView tv = tile_view(a, gm, ok);
    if (!ok) return;
    int64_t lo, hi;
    slot_chunk(tv, gm, lo, hi);
    const T* __restrict__ pcal = a.pcal + gm.uoff;
    const T* __restrict__ pobs = a.pobs + gm.uoff;
    double acc[NPART];
#pragma unroll
    for (int m = 0; m < NPART; ++m) acc[m] = 0.0;
    for (int64_t e = lo + tv.lane; e < hi; e += kUnroll * WAVE) {
        double pc[kUnroll], po[kUnroll];
        load_step(pcal, e, hi, pc);
        load_step(pobs, e, hi, po);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            if (e + (int64_t)u * WAVE >= hi) break;
            acc[0] += fpart(pc[u], po[u]);
            acc[1] += gpart(pc[u], po[u]);
            acc[2] += pc[u] - po[u];
        }
    }
    write_record(a.part, tv.slot, acc);
}

template <typename T>
__global__ __launch_bounds__(64) void k_decomp_mass(AuxArgs<T> a)
{
    const int g = blockIdx.x;
    const GatherMeta gm = a.meta[g];
    double q[NPART];
    reduce_records(a.part + (int64_t)gm.tile_base * NPART, gm.ntiles, q);
    if (threadIdx.x == 0) {
        a.mass_out[3 * g + 0] = gm.cm * q[0];
        a.mass_out[3 * g + 1] = gm.cm * q[1];
        a.mass_out[3 * g + 2] = q[2] / (double(gm.nr) * double(gm.nt));
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_decomp_source(AuxArgs<T> a)
{
    GatherMeta gm;
    bool ok;
    const TileView tv = tile_view(a, gm, ok);
    if (!ok) return;
    int64_t lo, hi;
    slot_chunk(tv, gm, lo, hi);
    const T* __restrict__ pcal = a.pcal + gm.uoff;
    const T* __restrict__ pobs = a.pobs + gm.uoff;
    T* __restrict__ s_out = a.s_out + gm.uoff;
    T* __restrict__ f_out = a.f_out ? a.f_out + gm.uoff : nullptr;
    T* __restrict__ g_out = a.g_out ? a.g_out + gm.uoff : nullptr;
    const double Mf = a.mass_out[3 * tv.g], Mg = a.mass_out[3 * tv.g + 1];
    const double mean = a.mass_out[3 * tv.g + 2];
    for (int64_t e = lo + tv.lane; e < hi; e += kUnroll * WAVE) {
        double pc[kUnroll], po[kUnroll];
        load_step(pcal, e, hi, pc);
        load_step(pobs, e, hi, po);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t k = e + (int64_t)u * WAVE;
            if (k >= hi) break;
            const double f = fpart(pc[u], po[u]), g = gpart(pc[u], po[u]);
            double s;
            if (a.mass_mode == MASS_BALANCE) s = (pc[u] - po[u]) - mean;
            else if (a.mass_mode == MASS_UNIT) s = (Mf > 0.0 ? f / Mf : 0.0) - (Mg > 0.0 ? g / Mg : 0.0);
            else s = pc[u] - po[u];
            s_out[k] = T(s);
            if (f_out) f_out[k] = T(f);
            if (g_out) g_out[k] = T(g);
        }
    }
}

// ------------------------------------------------------------------ adjoint

// partials: sum phi, <phi, f>, <phi, g>, sum f, sum g
template <typename T>
__global__ __launch_bounds__(256) void k_adj_sums(AuxArgs<T> a)
{
    GatherMeta gm;
    bool ok;
    const TileView tv = tile_view(a, gm, ok);
    if (!ok) return;
    int64_t lo, hi;
    slot_chunk(tv, gm, lo, hi);
    const T* __restrict__ phi = a.phi_user + gm.uoff;
    const bool unit = a.mass_mode == MASS_UNIT;
    const T* __restrict__ pcal = unit ? a.pcal + gm.uoff : nullptr;
    const T* __restrict__ pobs = unit ? a.pobs + gm.uoff : nullptr;
    double acc[NPART];
#pragma unroll
    for (int m = 0; m < NPART; ++m) acc[m] = 0.0;
    for (int64_t e = lo + tv.lane; e < hi; e += kUnroll * WAVE) {
        double ph[kUnroll], pc[kUnroll], po[kUnroll];
        load_step(phi, e, hi, ph);
        if (unit) {
            load_step(pcal, e, hi, pc);
            load_step(pobs, e, hi, po);
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            if (e + (int64_t)u * WAVE >= hi) break;
            acc[0] += ph[u];
            if (unit) {
                const double f = fpart(pc[u], po[u]), g = gpart(pc[u], po[u]);
                acc[1] += ph[u] * f;
                acc[2] += ph[u] * g;
                acc[3] += f;
                acc[4] += g;
            }
        }
    }
    write_record(a.part, tv.slot, acc);
}

// adj[4 g + 0] = scale dx dt gbar; [1] = mean phi (balance) or pf (unit); [2] = pg
template <typename T>
__global__ __launch_bounds__(64) void k_adj_scalars(AuxArgs<T> a)
{
    const int g = blockIdx.x;
    const GatherMeta gm = a.meta[g];
    double q[NPART];
    reduce_records(a.part + (int64_t)gm.tile_base * NPART, gm.ntiles, q);
    if (threadIdx.x == 0) {
        const double gb = a.gbar ? a.gbar[g] : 1.0;
        a.adj[4 * g + 0] = gm.cm * gb;
        if (a.mass_mode == MASS_BALANCE) {
            a.adj[4 * g + 1] = q[0] / (double(gm.nr) * double(gm.nt));
            a.adj[4 * g + 2] = 0.0;
        } else if (a.mass_mode == MASS_UNIT) {
            a.adj[4 * g + 1] = q[3] > 0.0 ? q[1] / q[3] : 0.0;
            a.adj[4 * g + 2] = q[4] > 0.0 ? q[2] / q[4] : 0.0;
        } else {
            a.adj[4 * g + 1] = 0.0;
            a.adj[4 * g + 2] = 0.0;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_adj_apply(AuxArgs<T> a)
{
    GatherMeta gm;
    bool ok;
    const TileView tv = tile_view(a, gm, ok);
    if (!ok) return;
    int64_t lo, hi;
    slot_chunk(tv, gm, lo, hi);
    const T* __restrict__ phi = a.phi_user + gm.uoff;
    const bool unit = a.mass_mode == MASS_UNIT;
    const T* __restrict__ pcal = unit ? a.pcal + gm.uoff : nullptr;
    T* __restrict__ psi = a.psi_out + gm.uoff;
    const double scale = a.adj[4 * tv.g], c1 = a.adj[4 * tv.g + 1], c2 = a.adj[4 * tv.g + 2];
    const double Mf = a.mass ? a.mass[3 * tv.g] : 0.0, Mg = a.mass ? a.mass[3 * tv.g + 1] : 0.0;
    for (int64_t e = lo + tv.lane; e < hi; e += kUnroll * WAVE) {
        double ph[kUnroll], pc[kUnroll];
        load_step(phi, e, hi, ph);
        if (unit) load_step(pcal, e, hi, pc);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t k = e + (int64_t)u * WAVE;
            if (k >= hi) break;
            double v;
            if (a.mass_mode == MASS_BALANCE) {
                v = scale * (ph[u] - c1);
            } else if (unit) {
                const double h = pc[u] > 0.0 ? 1.0 : 0.0;
                v = scale * ((Mf > 0.0 ? h * (ph[u] - c1) / Mf : 0.0) +
                             (Mg > 0.0 ? (1.0 - h) * (ph[u] - c2) / Mg : 0.0));
            } else {
                v = scale * ph[u];
            }
            psi[k] = T(v);
        }
    }
}

// ------------------------------------------------------------------ least squares

// psi = gbar dx dt (Pcal - Pobs) (optional); partial: sum (Pcal - Pobs)^2
template <typename T>
__global__ __launch_bounds__(256) void k_lsd_apply(AuxArgs<T> a)
{
    GatherMeta gm;
    bool ok;
    const TileView tv = tile_view(a, gm, ok);
    if (!ok) return;
    int64_t lo, hi;
    slot_chunk(tv, gm, lo, hi);
    const T* __restrict__ pcal = a.pcal + gm.uoff;
    const T* __restrict__ pobs = a.pobs + gm.uoff;
    T* __restrict__ psi = a.psi_out ? a.psi_out + gm.uoff : nullptr;
    const double scale = gm.cm * (a.gbar ? a.gbar[tv.g] : 1.0);
    double acc[NPART];
#pragma unroll
    for (int m = 0; m < NPART; ++m) acc[m] = 0.0;
    for (int64_t e = lo + tv.lane; e < hi; e += kUnroll * WAVE) {
        double pc[kUnroll], po[kUnroll];
        load_step(pcal, e, hi, pc);
        load_step(pobs, e, hi, po);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t k = e + (int64_t)u * WAVE;
            if (k >= hi) break;
            const double d = pc[u] - po[u];
            acc[0] = fma(d, d, acc[0]);
            if (psi) psi[k] = T(scale * d);
        }
    }
    write_record(a.part, tv.slot, acc);
}

// ------------------------------------------------------------------ grid transfer
//
// The multi-grid strategy: the EMD is first computed on a coarse grid, then the
// primal-dual method runs on the fine grid from the coarse solution.  The coarse
// grid groups fr receivers by ft samples, with spacings fr dx and ft dt, so the flux
// and the potential keep their scale between the grids.

// Restriction: coarse cell (I, J) = mean of the fine cells of its block (the last
// block of a row or column holds what is left).  A block walks coarse rows, its
// threads the samples of a row.
template <typename T>
__global__ __launch_bounds__(256) void k_restrict(XferArgs<T> a)
{
    const int g = blockIdx.y;
    const GatherMeta f = a.meta_f[g], c = a.meta_c[g];
    for (int I = blockIdx.x; I < c.nr; I += gridDim.x) {
        const int i0 = a.fr * I, i1 = min(i0 + a.fr, f.nr);
        const int64_t orow = c.uoff + (int64_t)I * c.nt;
        for (int J = threadIdx.x; J < c.nt; J += blockDim.x) {
            const int j0 = a.ft * J, j1 = min(j0 + a.ft, f.nt);
            double sum = 0.0;
            int count = 0;
            for (int i = i0; i < i1; ++i) {
                const T* row = a.in + f.uoff + (int64_t)i * f.nt;
                for (int j = j0; j < j1; ++j) {
                    sum += double(row[j]);
                    ++count;
                }
            }
            a.out[orow + J] = T(sum / count);
        }
    }
}

// Where fine index i falls between the coarse samples of one axis: samples k0, k1
// with weights w0, w1; k < 0 stands for a zero sample.  Cell-centred samples: the
// fine cell sits at coarse coordinate (i - (f - 1)/2) / f, clamped to [0, n - 1].
// Edge samples (a flux component along its own axis; edge k lies between cells
// k - 1 and k): fine edge i sits at i / f on the coarse edges 0..n, whose two ends
// are boundary edges carrying no flux.
struct AxisW {
    int k0, k1;
    double w0, w1;
};

__device__ __forceinline__ AxisW axis_w(int i, int f, int n, bool edge)
{
    const int hi = edge ? n : n - 1;
    double x = edge ? double(i) / f : (i - 0.5 * (f - 1)) / f;
    x = fmin(fmax(x, 0.0), double(hi));
    AxisW w;
    if (hi <= 0) {
        w.k0 = 0;
        w.k1 = 0;
        w.w0 = 1.0;
        w.w1 = 0.0;
    } else {
        int k = (int)floor(x);
        if (k >= hi) k = hi - 1;
        w.k0 = k;
        w.k1 = k + 1;
        w.w1 = x - k;
        w.w0 = 1.0 - w.w1;
    }
    if (edge) {
        if (w.k0 == 0 || w.k0 == n) w.k0 = -1;
        if (w.k1 == 0 || w.k1 == n) w.k1 = -1;
    }
    return w;
}

// The four coarse samples a bilinear weight pair reads (k < 0 stands for a zero
// sample).  Every load is made, at the gather's first element for a zero sample,
// and the zeros are chosen afterwards, so that all loads of a fine sample are in
// flight together instead of each behind a branch and a wait.
__device__ __forceinline__ int64_t cidx(const GatherMeta& c, int a, int b)
{
    return (a < 0 || b < 0) ? c.uoff : c.uoff + (int64_t)a * c.nt + b;
}

template <typename T>
__device__ __forceinline__ void load_quad(const T* v, const GatherMeta& c, const AxisW& r, const AxisW& t, T (&q)[4])
{
    q[0] = v[cidx(c, r.k0, t.k0)];
    q[1] = v[cidx(c, r.k0, t.k1)];
    q[2] = v[cidx(c, r.k1, t.k0)];
    q[3] = v[cidx(c, r.k1, t.k1)];
}

template <typename T>
__device__ __forceinline__ double cval(T x, int a, int b)
{
    return (a < 0 || b < 0) ? 0.0 : double(x);
}

template <typename T>
__device__ __forceinline__ double blend(const T (&q)[4], const AxisW& r, const AxisW& t)
{
    return r.w0 * t.w0 * cval(q[0], r.k0, t.k0) + r.w0 * t.w1 * cval(q[1], r.k0, t.k1) +
           r.w1 * t.w0 * cval(q[2], r.k1, t.k0) + r.w1 * t.w1 * cval(q[3], r.k1, t.k1);
}

// Prolongation: bilinear interpolation of the coarse u^x (receiver edges, time
// centres), u^t (time edges, receiver centres) and phi (centres) onto the fine
// grid.  The fine grid is cut into blocks of kProlongRows rows by 256 samples; a
// thread block takes them in turn, computes the rows' weights once into LDS, and each
// thread the weights of its sample once, then walks the rows.
constexpr int kProlongRows = 16;

template <typename T, bool HAS_U, bool HAS_PHI>
__global__ __launch_bounds__(256) void k_prolong(XferArgs<T> a)
{
    __shared__ AxisW rw[2][kProlongRows];  // [0]: cell centres, [1]: edges
    const int g = blockIdx.y;
    const GatherMeta f = a.meta_f[g], c = a.meta_c[g];
    const int strips = (f.nt + 255) / 256;
    const int pieces = strips * ((f.nr + kProlongRows - 1) / kProlongRows);
    for (int p = blockIdx.x; p < pieces; p += gridDim.x) {
        const int i0 = (p / strips) * kProlongRows;
        const int nrow = min(kProlongRows, f.nr - i0);
        const int j = (p % strips) * 256 + threadIdx.x;
        __syncthreads();  // the previous piece's rows have been read
        if (threadIdx.x < 2 * kProlongRows) {
            const int r = threadIdx.x % kProlongRows;
            const bool edge = threadIdx.x >= kProlongRows;
            if (r < nrow) rw[edge][r] = axis_w(i0 + r, a.fr, c.nr, edge);
        }
        __syncthreads();
        if (j >= f.nt) continue;
        const AxisW tc = axis_w(j, a.ft, c.nt, false), te = axis_w(j, a.ft, c.nt, true);
        const int64_t o0 = f.uoff + (int64_t)i0 * f.nt + j;
        for (int r = 0; r < nrow; ++r) {
            const AxisW rc = rw[0][r], re = rw[1][r];
            const int64_t o = o0 + (int64_t)r * f.nt;
            T qx[4], qt[4], qp[4];
            if constexpr (HAS_U) {
                load_quad(a.u_c, c, re, tc, qx);
                load_quad(a.u_c + a.len_c, c, rc, te, qt);
            }
            if constexpr (HAS_PHI) load_quad(a.phi_c, c, rc, tc, qp);
            if constexpr (HAS_U) {
                a.u_f[o] = T(blend(qx, re, tc));
                a.u_f[a.len_f + o] = T(blend(qt, rc, te));
            }
            if constexpr (HAS_PHI) a.phi_f[o] = T(blend(qp, rc, tc));
        }
    }
}

// value[g] = 1/2 dx dt sum (Pcal - Pobs)^2
template <typename T>
__global__ __launch_bounds__(64) void k_lsd_value(AuxArgs<T> a)
{
    const int g = blockIdx.x;
    const GatherMeta gm = a.meta[g];
    double q[NPART];
    reduce_records(a.part + (int64_t)gm.tile_base * NPART, gm.ntiles, q);
    if (threadIdx.x == 0) a.emd_out[g] = 0.5 * gm.cm * q[0];
}

// ------------------------------------------------------------------ plan-free decompose
//
// The same recombination and normalisation as k_decomp_*, for a batch described in
// the kernel arguments, with the per-gather sums in a scratch array the caller owns.
// Gather g is cut into kNdBlocks contiguous chunks of its nr * nt elements; block
// (b, g) sums chunk b (threads stride through it, the four waves' sums are added in
// order) into record (g, b), and one wave per gather adds its records in a fixed
// order: deterministic, and every record is rewritten by every call.

template <typename T>
__device__ __forceinline__ void nd_chunk(const NdArgs<T>& a, int g, int b, int64_t& lo, int64_t& hi)
{
    const int64_t n = a.g[g].n;
    const int64_t chunk = (n + kNdBlocks - 1) / kNdBlocks;
    lo = min((int64_t)b * chunk, n);
    hi = min(lo + chunk, n);
}

template <typename T>
__global__ __launch_bounds__(256) void k_nd_sums(NdArgs<T> a)
{
    const int g = blockIdx.y, b = blockIdx.x;
    int64_t lo, hi;
    nd_chunk(a, g, b, lo, hi);
    const int64_t off = a.g[g].off;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t e = lo + threadIdx.x; e < hi; e += blockDim.x) {
        const double pc = double(a.pcal[off + e]), po = double(a.pobs[off + e]);
        acc[0] += fpart(pc, po);
        acc[1] += gpart(pc, po);
        acc[2] += pc - po;
    }
    __shared__ double red[4][3];
    const int w = threadIdx.x / WAVE;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const double v = wave_sum(acc[q]);
        if ((threadIdx.x & (WAVE - 1)) == 0) red[w][q] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double* rec = a.scratch + ((int64_t)g * kNdBlocks + b) * 3;
#pragma unroll
        for (int q = 0; q < 3; ++q) rec[q] = ((red[0][q] + red[1][q]) + red[2][q]) + red[3][q];
    }
}

template <typename T>
__global__ __launch_bounds__(64) void k_nd_mass(NdArgs<T> a)
{
    const int g = blockIdx.x;
    const int lane = threadIdx.x;
    const double* rec = a.scratch + (int64_t)g * kNdBlocks * 3;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int b = lane; b < kNdBlocks; b += WAVE) {
#pragma unroll
        for (int q = 0; q < 3; ++q) acc[q] += rec[b * 3 + q];
    }
    double sum[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) sum[q] = wave_sum(acc[q]);
    if (lane == 0) {
        a.mass_out[3 * g + 0] = a.g[g].cm * sum[0];
        a.mass_out[3 * g + 1] = a.g[g].cm * sum[1];
        a.mass_out[3 * g + 2] = sum[2] / double(a.g[g].n);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_nd_source(NdArgs<T> a)
{
    const int g = blockIdx.y, b = blockIdx.x;
    int64_t lo, hi;
    nd_chunk(a, g, b, lo, hi);
    const int64_t off = a.g[g].off;
    const double Mf = a.mass_out[3 * g], Mg = a.mass_out[3 * g + 1], mean = a.mass_out[3 * g + 2];
    for (int64_t e = lo + threadIdx.x; e < hi; e += blockDim.x) {
        const double pc = double(a.pcal[off + e]), po = double(a.pobs[off + e]);
        const double f = fpart(pc, po), gg = gpart(pc, po);
        double s;
        if (a.mass_mode == MASS_BALANCE) s = (pc - po) - mean;
        else if (a.mass_mode == MASS_UNIT) s = (Mf > 0.0 ? f / Mf : 0.0) - (Mg > 0.0 ? gg / Mg : 0.0);
        else s = pc - po;
        a.s_out[off + e] = T(s);
        if (a.f_out) a.f_out[off + e] = T(f);
        if (a.g_out) a.g_out[off + e] = T(gg);
    }
}

}  // namespace

template <typename T>
void launch_decompose_noalloc(const NdArgs<T>& a, hipStream_t stream)
{
    hipLaunchKernelGGL(k_nd_sums<T>, dim3(kNdBlocks, a.ngather), dim3(256), 0, stream, a);
    hipLaunchKernelGGL(k_nd_mass<T>, dim3(a.ngather), dim3(64), 0, stream, a);
    hipLaunchKernelGGL(k_nd_source<T>, dim3(kNdBlocks, a.ngather), dim3(256), 0, stream, a);
}

template <typename T>
void launch_lsd(const AuxArgs<T>& a, int grid, hipStream_t stream)
{
    hipLaunchKernelGGL(k_lsd_apply<T>, dim3(grid), dim3(256), 0, stream, a);
    hipLaunchKernelGGL(k_lsd_value<T>, dim3(a.ngather), dim3(64), 0, stream, a);
}

template <typename T>
void launch_copy_in(const AuxArgs<T>& a, int warm, int grid, hipStream_t stream)
{
    hipLaunchKernelGGL(k_copy_in<T>, dim3(grid), dim3(256), 0, stream, a, warm);
}

template <typename T>
void launch_gather_init(const AuxArgs<T>& a, hipStream_t stream)
{
    hipLaunchKernelGGL(k_gather_init<T>, dim3(a.ngather), dim3(64), 0, stream, a);
}

template <typename T>
void launch_copy_out(const AuxArgs<T>& a, int grid, hipStream_t stream)
{
    hipLaunchKernelGGL(k_copy_out<T>, dim3(grid), dim3(256), 0, stream, a);
}

template <typename T>
void launch_finalize(const AuxArgs<T>& a, int grid, hipStream_t stream)
{
    hipLaunchKernelGGL(k_lagr_sums<T>, dim3(grid), dim3(256), 0, stream, a);
    hipLaunchKernelGGL(k_finalize<T>, dim3(a.ngather), dim3(64), 0, stream, a);
}

template <typename T>
void launch_decompose(const AuxArgs<T>& a, int grid, hipStream_t stream)
{
    hipLaunchKernelGGL(k_decomp_sums<T>, dim3(grid), dim3(256), 0, stream, a);
    hipLaunchKernelGGL(k_decomp_mass<T>, dim3(a.ngather), dim3(64), 0, stream, a);
    hipLaunchKernelGGL(k_decomp_source<T>, dim3(grid), dim3(256), 0, stream, a);
}

template <typename T>
void launch_adjoint(const AuxArgs<T>& a, int grid, hipStream_t stream)
{
    hipLaunchKernelGGL(k_adj_sums<T>, dim3(grid), dim3(256), 0, stream, a);
    hipLaunchKernelGGL(k_adj_scalars<T>, dim3(a.ngather), dim3(64), 0, stream, a);
    hipLaunchKernelGGL(k_adj_apply<T>, dim3(grid), dim3(256), 0, stream, a);
}

template <typename T>
void launch_restrict(const XferArgs<T>& a, int ngather, int blocks, hipStream_t stream)
{
    hipLaunchKernelGGL(k_restrict<T>, dim3(blocks, ngather), dim3(256), 0, stream, a);
}

template <typename T>
void launch_prolong(const XferArgs<T>& a, int ngather, int blocks, hipStream_t stream)
{
    // one kernel per set of outputs, so that no branch separates a row's loads
    if (a.u_f && a.phi_f)
        hipLaunchKernelGGL((k_prolong<T, true, true>), dim3(blocks, ngather), dim3(256), 0, stream, a);
    else if (a.u_f)
        hipLaunchKernelGGL((k_prolong<T, true, false>), dim3(blocks, ngather), dim3(256), 0, stream, a);
    else
        hipLaunchKernelGGL((k_prolong<T, false, true>), dim3(blocks, ngather), dim3(256), 0, stream, a);
}

void launch_zero_counter(int32_t* counter, hipStream_t stream)
{
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, stream, counter);
}

#define EMD_INST(T)                                                                  \
    template void launch_copy_in<T>(const AuxArgs<T>&, int, int, hipStream_t);      \
    template void launch_gather_init<T>(const AuxArgs<T>&, hipStream_t);            \
    template void launch_copy_out<T>(const AuxArgs<T>&, int, hipStream_t);          \
    template void launch_finalize<T>(const AuxArgs<T>&, int, hipStream_t);          \
    template void launch_decompose<T>(const AuxArgs<T>&, int, hipStream_t);         \
    template void launch_adjoint<T>(const AuxArgs<T>&, int, hipStream_t);           \
    template void launch_lsd<T>(const AuxArgs<T>&, int, hipStream_t);                \
    template void launch_restrict<T>(const XferArgs<T>&, int, int, hipStream_t);     \
    template void launch_prolong<T>(const XferArgs<T>&, int, int, hipStream_t);     \
    template void launch_decompose_noalloc<T>(const NdArgs<T>&, hipStream_t);
EMD_INST(float)
EMD_INST(double)
#undef EMD_INST

}  // namespace emd
