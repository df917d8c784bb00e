// emd_abi.hip -- host implementation of the C ABI declared in include/emd_mi355x.h.
//
// A plan owns the solver workspace for one batch of gathers: the padded,
// double-buffered solver fields, the tile table, per-gather metadata and scalar
// state, and the reduction partials.  emd_pdhg_solve enqueues one fused sweep per
// PDHG iteration for the whole batch (replayed from a captured HIP graph in chunks
// of sweeps_per_sync launches) and reads the finished-gather count between chunks.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cstddef>
#include <mutex>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "emd_internal.h"
#include "emd_launch.h"
#include "emd_mi355x.h"

using namespace emd;

namespace {

thread_local std::string g_last_error;

emd_status fail(emd_status st, const std::string& msg)
{
    g_last_error = msg;
    return st;
}

#define HIP_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(EMD_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));     \
    } while (0)

// A named host range around each compute call, seen by rocprofv3 --marker-trace
// (a no-op when no tool is attached).
struct Range {
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};

constexpr int kWavesPerBlock = tiling::kWavesPerBlock;
constexpr int kDefaultRows = 16;
constexpr int kChains = 2;  // independent chains of sweep launches per captured chunk

using tiling::round_up;

}  // namespace

struct emd_plan {
    int device = -1;
    int32_t ngather = 0;
    int64_t batch_len = 0;
    emd_params params{};
    std::vector<emd_gather_desc> desc;
    size_t elem = 4;          // bytes per field element
    int vec = 4;              // elements per lane vector
    int rows = kDefaultRows;  // receiver rows per tile (the default for every gather)
    std::vector<int> grows;   // receiver rows per tile, per gather
    int64_t padded_len = 0;
    int32_t ntiles = 0;       // entries of the tile table (including empty padding)
    int32_t nslots = 0;       // real tiles = partial-sum slots
    int grid = 0;             // blocks per tile-table launch (multiple of 8)
    int64_t cells = 0;

    // host copy of the tiling: per-gather metadata, time tiles and row strips
    std::vector<GatherMeta> h_meta;
    std::vector<int> h_ntt, h_nst;

    // device memory
    GatherMeta* d_meta = nullptr;
    Tile* d_tiles = nullptr;      // every gather's tiles (auxiliary kernels, first chunk)
    Tile* d_tiles_act = nullptr;  // [kChains][act_cap] the running gathers' tiles, by chain
    int64_t act_cap = 0;          // entries per chain in d_tiles_act
    void* d_fields = nullptr;  // one allocation: s, ux[2], ut[2], phi[2], R[2]
    double* d_part = nullptr;     // [2][slots][NPART]
    double* d_part_l1 = nullptr;  // [2][slots][NPART_L1] (l1 linesearch test)
    GState* d_gst = nullptr;   // [2][ngather]
    int32_t* d_done = nullptr;
    double* d_adj = nullptr;   // [ngather][4]
    ResumeRec* d_resume = nullptr;  // [ngather] checkpoint a resumed solve continues from
    std::vector<GState> last_state;  // per-gather state at the end of the last solve
    bool state_on_device = false;    // the last solve (fixed budget) has not been read back
    std::vector<int32_t> resume_iters;  // its checkpointed iteration counts (resume), or empty
    int32_t* h_done = nullptr; // pinned
    int64_t workspace_bytes = 0;

    // captured chunk of sweeps (rebuilt when the arguments change)
    hipGraphExec_t graph = nullptr;
    int graph_chunk = 0;
    std::vector<unsigned char> graph_key;

    double* d_hist = nullptr;  // caller's residual-history ring, or NULL
    int32_t hist_cap = 0;

    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int64_t last_sweeps = 0;
    int64_t last_cell_updates = 0;
    int64_t last_rebuilds = 0;
    bool timing_valid = false;
    std::vector<emd_gather_desc> host_meta_cache;
};

namespace {

emd_status check_device(emd_plan* plan)
{
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (plan && dev != plan->device)
        return fail(EMD_ERR_DEVICE, "current device differs from the plan's device");
    return EMD_SUCCESS;
}

emd_status validate_params(const emd_params* p)
{
    if (!p) return fail(EMD_ERR_NULL_POINTER, "params is NULL");
    auto bad = [](const char* what) { return fail(EMD_ERR_INVALID_ARGUMENT, what); };
    if (!(p->eps >= 0.0) || !std::isfinite(p->eps)) return bad("eps must be finite and >= 0");
    if (!(p->xi > 0.0 && p->xi < 1.0)) return bad("xi must lie in (0, 1)");
    if (!(p->zeta > 0.0 && p->zeta < 1.0)) return bad("zeta must lie in (0, 1)");
    if (!(p->delta > 0.0) || !std::isfinite(p->delta)) return bad("delta must be finite and > 0");
    if (!std::isfinite(p->alpha1)) return bad("alpha1 must be finite");
    if (!std::isfinite(p->alpha_max_factor)) return bad("alpha_max_factor must be finite");
    if (!(p->tol_res >= 0.0)) return bad("tol_res must be >= 0");
    if (!(p->mass_tol >= 0.0)) return bad("mass_tol must be >= 0");
    if (p->max_iter < 1) return bad("max_iter must be >= 1");
    if (p->check_every < 1) return bad("check_every must be >= 1");
    if (p->max_ls_trials < 0 || p->max_ls_trials > 1000) return bad("max_ls_trials must lie in [0, 1000]");
    if (p->ls_mode < EMD_LS_L2 || p->ls_mode > EMD_LS_FIXED) return bad("unknown ls_mode");
    if (p->mass_mode < EMD_MASS_BALANCE || p->mass_mode > EMD_MASS_NONE) return bad("unknown mass_mode");
    if (p->precision != EMD_F32 && p->precision != EMD_F64) return bad("unknown precision");
    // a solve reads the newest state from buffer 0, so every chunk is an even number
    // of sweeps; 0 selects the fixed-budget solve (no reads between sweeps)
    if (p->iters_per_sweep < 0 || p->iters_per_sweep > 3) return bad("iters_per_sweep must be 0, 1, 2 or 3");
    if (p->iters_per_sweep >= 2 && p->ls_mode != EMD_LS_FIXED)
        return bad("two or three iterations per sweep need fixed steps (ls_mode EMD_LS_FIXED)");
    if (p->iters_per_sweep >= 2 && p->check_every % p->iters_per_sweep != 0)
        return bad("K iterations per sweep check the stop rule on multiples of K: check_every must be one");
    // a sweep of K iterations reaches K samples past its tile in time, which the halo
    // lanes carry: four FP32 samples each, two FP64 ones
    if (p->iters_per_sweep == 3 && p->precision == EMD_F64)
        return bad("three iterations per sweep need FP32 fields (an FP64 lane carries two halo samples)");
    if (p->sweeps_per_sync != 0 &&
        (p->sweeps_per_sync < 2 || p->sweeps_per_sync > 4096 || (p->sweeps_per_sync & 1)))
        return bad("sweeps_per_sync must be 0, or even and in [2, 4096]");
    return EMD_SUCCESS;
}

void destroy_graph(emd_plan* plan)
{
    if (plan->graph) {
        (void)hipGraphExecDestroy(plan->graph);
        plan->graph = nullptr;
    }
    plan->graph_key.clear();
    plan->graph_chunk = 0;
}

// The tile table of the selected gathers, laid out over the XCDs (emd_tiling.h).
std::vector<Tile> layout_tiles(const emd_plan* plan, const std::vector<char>& sel)
{
    tiling::Layout L;
    L.meta = plan->h_meta;
    L.ntt = plan->h_ntt;
    L.nst = plan->h_nst;
    return tiling::layout_tiles(L, OUT_LANES * plan->vec, sel);
}

// Device memory a plan owns: the nine padded field copies, the scalar state, the
// partial-sum slots of both linesearch forms, the tile tables and the metadata.
int64_t plan_workspace_bytes(const emd_plan* plan)
{
    return (int64_t)plan->elem * plan->padded_len * 9 + (int64_t)sizeof(GState) * 2 * plan->ngather +
           (int64_t)sizeof(double) * (NPART + NPART_L1) * 2 * plan->nslots +
           (int64_t)sizeof(Tile) * (1 + 2 * kChains) * plan->ntiles +
           (int64_t)sizeof(GatherMeta) * plan->ngather;
}

emd_status build_tiles(emd_plan* plan)
{
    const int span = OUT_LANES * plan->vec;
    std::vector<tiling::GatherIn> gin(plan->ngather);
    for (int g = 0; g < plan->ngather; ++g) {
        const emd_gather_desc& d = plan->desc[g];
        gin[g] = tiling::GatherIn{d.nr, d.nt, d.dx, d.dt, d.offset, plan->grows[g]};
    }
    const tiling::Layout L = tiling::plan_layout(gin, span, plan->params.alpha1, plan->params.delta);
    const std::vector<GatherMeta>& meta = L.meta;
    const int32_t slots = L.slots;
    const int64_t poff = L.padded_len;
    plan->h_meta = meta;
    plan->h_ntt = L.ntt;
    plan->h_nst = L.nst;
    const std::vector<Tile> tiles = layout_tiles(plan, std::vector<char>(plan->ngather, 1));
    if (tiles.size() > (size_t)INT32_MAX / 8) return fail(EMD_ERR_INVALID_ARGUMENT, "too many tiles");
    const bool realloc_tiles = (int32_t)tiles.size() != plan->ntiles || slots != plan->nslots || !plan->d_tiles;
    plan->ntiles = (int32_t)tiles.size();
    plan->nslots = slots;
    plan->padded_len = poff;
    plan->grid = (int)(tiles.size() / kWavesPerBlock);  // kXcd runs of whole blocks
    plan->act_cap = 2 * (int64_t)tiles.size();
    if (realloc_tiles) {
        if (plan->d_tiles) (void)hipFree(plan->d_tiles);
        if (plan->d_tiles_act) (void)hipFree(plan->d_tiles_act);
        if (plan->d_part) (void)hipFree(plan->d_part);
        if (plan->d_part_l1) (void)hipFree(plan->d_part_l1);
        plan->d_tiles = nullptr;
        plan->d_tiles_act = nullptr;
        plan->d_part = nullptr;
        plan->d_part_l1 = nullptr;
        if (hipMalloc(&plan->d_tiles, sizeof(Tile) * tiles.size()) != hipSuccess ||
            hipMalloc(&plan->d_tiles_act, sizeof(Tile) * 2 * tiles.size() * kChains) != hipSuccess ||
            hipMalloc(&plan->d_part, sizeof(double) * NPART * 2 * slots) != hipSuccess ||
            hipMalloc(&plan->d_part_l1, sizeof(double) * NPART_L1 * 2 * slots) != hipSuccess)
            return fail(EMD_ERR_OUT_OF_MEMORY, "cannot allocate the tile table");
    }
    if (!plan->d_meta && hipMalloc(&plan->d_meta, sizeof(GatherMeta) * plan->ngather) != hipSuccess)
        return fail(EMD_ERR_OUT_OF_MEMORY, "cannot allocate gather metadata");
    HIP_TRY(hipMemcpy(plan->d_tiles, tiles.data(), sizeof(Tile) * tiles.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(plan->d_meta, meta.data(), sizeof(GatherMeta) * meta.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(plan->d_part, 0, sizeof(double) * NPART * 2 * slots));
    HIP_TRY(hipMemset(plan->d_part_l1, 0, sizeof(double) * NPART_L1 * 2 * slots));
    destroy_graph(plan);
    plan->workspace_bytes = plan_workspace_bytes(plan);
    return EMD_SUCCESS;
}

template <typename T>
T* field(emd_plan* plan, int k)
{
    return reinterpret_cast<T*>(plan->d_fields) + (int64_t)k * plan->padded_len;
}

SolveScalars scalars(const emd_plan* plan, int ls_mode, const double* replay, int ld_replay)
{
    SolveScalars sc;
    sc.eps = plan->params.eps;
    sc.xi = plan->params.xi;
    sc.zeta = plan->params.zeta;
    sc.delta = plan->params.delta;
    sc.tol_res = plan->params.tol_res;
    sc.max_iter = plan->params.max_iter;
    sc.check_every = plan->params.check_every;
    sc.max_ls_trials = plan->params.max_ls_trials;
    sc.ls_mode = ls_mode;
    sc.replay = replay;
    sc.ld_replay = ld_replay;
    sc.pad = 0;
    sc.hist = plan->d_hist;
    sc.hist_cap = plan->hist_cap;
    sc.pad2 = 0;
    return sc;
}

template <typename T>
AuxArgs<T> aux_args(emd_plan* plan)
{
    AuxArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    a.meta = plan->d_meta;
    a.tiles = plan->d_tiles;
    a.ntiles = plan->ntiles;
    a.ngather = plan->ngather;
    a.mass_mode = plan->params.mass_mode;
    a.mass_tol = plan->params.mass_tol;
    a.batch_len = plan->batch_len;
    a.s_pad = field<T>(plan, 0);
    for (int b = 0; b < 2; ++b) {
        a.ux[b] = field<T>(plan, 1 + b);
        a.ut[b] = field<T>(plan, 3 + b);
        a.phi[b] = field<T>(plan, 5 + b);
        a.R[b] = field<T>(plan, 7 + b);
    }
    a.part = plan->d_part;
    a.gst = plan->d_gst;
    a.done = plan->d_done;
    a.adj = plan->d_adj;
    a.eps = plan->params.eps;
    a.alpha_max_factor = plan->params.alpha_max_factor;
    return a;
}

template <typename T>
SweepArgs<T> sweep_args(emd_plan* plan, const SolveScalars& sc)
{
    SweepArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    a.meta = plan->d_meta;
    a.tiles = plan->d_tiles;
    a.ntiles = plan->ntiles;
    a.s = field<T>(plan, 0);
    for (int b = 0; b < 2; ++b) {
        a.ux[b] = field<T>(plan, 1 + b);
        a.ut[b] = field<T>(plan, 3 + b);
        a.phi[b] = field<T>(plan, 5 + b);
        a.R[b] = field<T>(plan, 7 + b);
        a.part[b] = sc.ls_mode == LS_L1 ? plan->d_part_l1 + (int64_t)b * plan->nslots * NPART_L1
                                        : plan->d_part + (int64_t)b * plan->nslots * NPART;
        a.gst[b] = plan->d_gst + (int64_t)b * plan->ngather;
    }
    a.done = plan->d_done;
    a.l1 = sc.ls_mode == LS_L1;
    a.ips = sc.ls_mode == LS_FIXED && plan->params.iters_per_sweep >= 2 ? plan->params.iters_per_sweep : 0;
    a.sc = sc;
    return a;
}

// The sweep launches of a solve.  The running gathers are split into up to kChains
// groups of about equal cells (one group once they hold fewer than
// tiling::kChainMinTiles tiles), each with its own tile table (laid out over the XCDs
// like the full table), and a captured chunk runs the groups as independent chains
// of launches: while the last waves of one group's sweep drain, the other group's
// next sweep fills the GPU.  A gather belongs to exactly one chain, so its sweeps
// stay in order; the groups share nothing but the finished counter.
template <typename T>
struct Chains {
    int n;
    int grid[kChains];
    SweepArgs<T> args[kChains];
};

// Split the selected gathers (largest first, each to the lighter group) and upload
// the groups' tile tables.  Falls back to one chain over the full table when a
// group's table would not fit its share of the buffer.
template <typename T>
emd_status build_chains(emd_plan* plan, const std::vector<char>& sel, const SweepArgs<T>& base,
                        Chains<T>& ch, hipStream_t stream)
{
    std::memset(&ch, 0, sizeof(ch));  // the graph key compares these bytes
    std::vector<int64_t> cells(plan->ngather);
    for (int g = 0; g < plan->ngather; ++g) cells[g] = (int64_t)plan->desc[g].nr * plan->desc[g].nt;
    int64_t sel_tiles = 0;
    for (int g = 0; g < plan->ngather; ++g)
        if (sel[g]) sel_tiles += plan->h_meta[g].ntiles;
    const std::vector<std::vector<char>> part =
        tiling::split_chains(cells, sel, tiling::chain_count(sel_tiles, kChains));
    const int nc = (int)part.size();
    std::vector<std::vector<Tile>> tabs(nc);
    for (int k = 0; k < nc; ++k) {
        tabs[k] = layout_tiles(plan, part[k]);
        if ((int64_t)tabs[k].size() > plan->act_cap) {
            ch.n = 1;
            ch.args[0] = base;
            ch.args[0].tiles = plan->d_tiles;
            ch.args[0].ntiles = plan->ntiles;
            ch.grid[0] = plan->grid;
            return EMD_SUCCESS;
        }
    }
    ch.n = nc;
    for (int k = 0; k < nc; ++k) {
        Tile* dst = plan->d_tiles_act + (int64_t)k * plan->act_cap;
        HIP_TRY(hipMemcpyAsync(dst, tabs[k].data(), sizeof(Tile) * tabs[k].size(), hipMemcpyHostToDevice, stream));
        ch.args[k] = base;
        ch.args[k].tiles = dst;
        ch.args[k].ntiles = (int32_t)tabs[k].size();
        ch.grid[k] = (int)(tabs[k].size() / kWavesPerBlock);
    }
    HIP_TRY(hipStreamSynchronize(stream));  // the host tables must outlive the copies
    return EMD_SUCCESS;
}

// Read the per-gather state the last solve left in buffer 0 and derive the plan
// statistics from it: cell updates = sum of nr nt times the iterations the solve ran
// (past a resumed checkpoint's).  wait: the solve's stream is not known to be done
// (a fixed-budget solve, possibly replayed from a caller's graph), so the device is
// synchronised first.
emd_status read_state(emd_plan* plan, bool wait)
{
    if (!plan->state_on_device) return EMD_SUCCESS;
    if (wait) HIP_TRY(hipDeviceSynchronize());
    std::vector<GState> st(plan->ngather);
    HIP_TRY(hipMemcpy(st.data(), plan->d_gst, sizeof(GState) * plan->ngather, hipMemcpyDeviceToHost));
    int64_t cu = 0;
    for (int g = 0; g < plan->ngather; ++g) {
        const int64_t it0 = !plan->resume_iters.empty() && st[g].status != ST_ZERO_SOURCE ? plan->resume_iters[g] : 0;
        cu += (int64_t)plan->desc[g].nr * plan->desc[g].nt * std::max<int64_t>(st[g].iters - it0, 0);
    }
    plan->last_cell_updates = cu;
    plan->last_state = st;
    plan->state_on_device = false;
    return EMD_SUCCESS;
}

// Enqueue `count` (even) sweeps starting at parity 0.  Uses a captured graph of
// sweeps_per_sync launches per chain when count equals that chunk size.
template <typename T>
emd_status enqueue_sweeps(emd_plan* plan, const Chains<T>& ch, int count, hipStream_t stream)
{
    const int chunk = plan->params.sweeps_per_sync;
    if (count == chunk) {
        std::vector<unsigned char> key(sizeof(ch));
        std::memcpy(key.data(), &ch, sizeof(ch));
        if (!plan->graph || plan->graph_chunk != chunk || plan->graph_key != key) {
            destroy_graph(plan);
            hipStream_t cs[kChains] = {};
            hipEvent_t fork = nullptr, join[kChains] = {};
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamCreateWithFlags(&cs[0], hipStreamNonBlocking);
            for (int k = 1; k < ch.n && e == hipSuccess; ++k) {
                e = hipStreamCreateWithFlags(&cs[k], hipStreamNonBlocking);
                if (e == hipSuccess) e = hipEventCreateWithFlags(&join[k], hipEventDisableTiming);
            }
            if (e == hipSuccess) e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
            if (e == hipSuccess) e = hipStreamBeginCapture(cs[0], hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                // fork the other chains off the capture stream, join them at the end
                if (ch.n > 1) (void)hipEventRecord(fork, cs[0]);
                for (int k = 1; k < ch.n; ++k) (void)hipStreamWaitEvent(cs[k], fork, 0);
                for (int n = 0; n < count; ++n)
                    for (int k = 0; k < ch.n; ++k) launch_sweep<T>(ch.args[k], n & 1, ch.grid[k], cs[k]);
                for (int k = 1; k < ch.n; ++k) {
                    (void)hipEventRecord(join[k], cs[k]);
                    (void)hipStreamWaitEvent(cs[0], join[k], 0);
                }
                e = hipStreamEndCapture(cs[0], &g);
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&plan->graph, g, nullptr, nullptr, 0);
            if (g) (void)hipGraphDestroy(g);
            if (fork) (void)hipEventDestroy(fork);
            for (int k = 0; k < kChains; ++k) {
                if (join[k]) (void)hipEventDestroy(join[k]);
                if (cs[k]) (void)hipStreamDestroy(cs[k]);
            }
            if (e != hipSuccess) {
                plan->graph = nullptr;
                return fail(EMD_ERR_HIP, std::string("graph capture of the sweeps failed: ") +
                                             hipGetErrorString(e));
            }
            plan->graph_chunk = chunk;
            plan->graph_key = key;
        }
        HIP_TRY(hipGraphLaunch(plan->graph, stream));
        return EMD_SUCCESS;
    }
    for (int n = 0; n < count; ++n)
        for (int k = 0; k < ch.n; ++k) launch_sweep<T>(ch.args[k], n & 1, ch.grid[k], stream);
    HIP_TRY(hipGetLastError());
    return EMD_SUCCESS;
}

template <typename T>
emd_status solve_impl(emd_plan* plan, const void* s, void* u, void* phi, int warm,
                      const double* d_mass, const double* replay, int ld_replay, double* d_emd,
                      emd_solve_info* d_info, hipStream_t stream, const ResumeRec* h_resume = nullptr)
{
    if (h_resume)
        HIP_TRY(hipMemcpyAsync(plan->d_resume, h_resume, sizeof(ResumeRec) * plan->ngather,
                               hipMemcpyHostToDevice, stream));
    AuxArgs<T> a = aux_args<T>(plan);
    a.s_user = static_cast<const T*>(s);
    a.u_user_in = warm ? static_cast<const T*>(u) : nullptr;
    a.phi_user_in = warm ? static_cast<const T*>(phi) : nullptr;
    a.u_user_out = static_cast<T*>(u);
    a.phi_user_out = static_cast<T*>(phi);
    a.mass = d_mass;
    a.emd_out = d_emd;
    a.info_out = d_info;
    a.resume = h_resume ? plan->d_resume : nullptr;

    launch_zero_counter(plan->d_done, stream);
    launch_copy_in<T>(a, warm, plan->grid, stream);
    launch_gather_init<T>(a, stream);
    HIP_TRY(hipGetLastError());

    const int ls_mode = replay ? LS_REPLAY : plan->params.ls_mode;
    const SweepArgs<T> sa = sweep_args<T>(plan, scalars(plan, ls_mode, replay, ld_replay));
    const int chunk = plan->params.sweeps_per_sync;
    // a gather needs iters + 1 sweeps, the last one applying the final dual step;
    // the l1 test may add an evaluation sweep per NL1 failed backtracking trials
    const int64_t evals = ls_mode == LS_L1 ? plan->params.max_ls_trials / NL1 + 1 : 0;
    // K iterations per sweep: ceil(max_iter / K) sweeps of work (one more to align a
    // resumed count that is not a multiple of K), then the sweep that takes the last
    // decision
    const int64_t K = sa.ips;
    const int64_t max_sweeps = K ? round_up(((int64_t)plan->params.max_iter + K - 1) / K + 2, 2)
                                 : round_up(((int64_t)plan->params.max_iter + 2) * (1 + evals), 2);
    plan->resume_iters.clear();
    if (h_resume)
        for (int g = 0; g < plan->ngather; ++g) plan->resume_iters.push_back(h_resume[g].iters);
    if (chunk == 0) {
        // Fixed budget: every sweep the budget allows goes on the stream, over the full
        // tile table, with nothing read back (the stop rule still ends each gather's
        // iterations on the device; its later sweeps only carry its state).  The same
        // tiles and slots as the chunked solve, so the same bits.  Nothing here
        // synchronises or allocates, so a caller can capture the call into a graph.
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        HIP_TRY(hipStreamIsCapturing(stream, &cap));
        const bool timed = cap == hipStreamCaptureStatusNone;
        if (timed) HIP_TRY(hipEventRecord(plan->ev0, stream));
        for (int64_t n = 0; n < max_sweeps; ++n) launch_sweep<T>(sa, (int)(n & 1), plan->grid, stream);
        if (timed) HIP_TRY(hipEventRecord(plan->ev1, stream));
        HIP_TRY(hipGetLastError());
        plan->last_sweeps = max_sweeps;
        plan->last_rebuilds = 0;
        plan->timing_valid = timed;
        a.gst = plan->d_gst;
        launch_finalize<T>(a, plan->grid, stream);
        launch_copy_out<T>(a, plan->grid, stream);
        HIP_TRY(hipGetLastError());
        plan->state_on_device = true;  // read back when the state or statistics are asked for
        return EMD_SUCCESS;
    }
    Chains<T> ch;
    std::memset(&ch, 0, sizeof(ch));
    std::vector<char> sel(plan->ngather, 1);
    emd_status cst = build_chains<T>(plan, sel, sa, ch, stream);
    if (cst != EMD_SUCCESS) return cst;
    int64_t sweeps = 0;
    // Finished gathers leave the sweep's tile tables: once the running gathers hold at
    // most 15/16 of the tables' cells, the chains are rebuilt from them alone and spread
    // over the XCDs again.  Tiles keep their shape and partial-sum slots, so every
    // decision, and hence every result, is bitwise the same as with the full table.
    int64_t table_cells = plan->cells;
    int32_t known_out = 0;  // finished gathers seen at the last status read
    int64_t rebuilds = 0;
    std::vector<GState> gs(plan->ngather);
    HIP_TRY(hipEventRecord(plan->ev0, stream));
    for (;;) {
        // the finished count before any sweep (gathers with nothing to solve)
        HIP_TRY(hipMemcpyAsync(plan->h_done, plan->d_done, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        const int32_t done = *plan->h_done;
        if (done >= plan->ngather || sweeps >= max_sweeps) break;
        if (sweeps > 0 && done > known_out) {
            // Every chunk has an even number of sweeps, so buffer 0 holds the newest
            // state and buffer 1 the state one sweep older (before the first sweep
            // buffer 1 still holds a previous solve's state).  A gather already
            // finished in buffer 1 has had its final state carried into both, and
            // stays correct after it stops being swept.
            HIP_TRY(hipMemcpyAsync(gs.data(), plan->d_gst + plan->ngather, sizeof(GState) * plan->ngather,
                                   hipMemcpyDeviceToHost, stream));
            HIP_TRY(hipStreamSynchronize(stream));
            int64_t live = 0;
            int32_t out = 0;
            for (int g = 0; g < plan->ngather; ++g) {
                sel[g] = gs[g].status == ST_RUNNING;
                if (sel[g]) live += (int64_t)plan->desc[g].nr * plan->desc[g].nt;
                else ++out;
            }
            known_out = out;
            if (tiling::narrow_now(live, table_cells)) {
                cst = build_chains<T>(plan, sel, sa, ch, stream);
                if (cst != EMD_SUCCESS) return cst;
                table_cells = live;
                ++rebuilds;
                const std::string mark = "emd: sweep tables narrowed after " + std::to_string(sweeps) +
                                         " sweeps, running gathers: " +
                                         std::to_string(plan->ngather - out);
                roctxMarkA(mark.c_str());
            }
        }
        const int count = (int)std::min<int64_t>(chunk, max_sweeps - sweeps);
        emd_status st = enqueue_sweeps<T>(plan, ch, count, stream);
        if (st != EMD_SUCCESS) return st;
        sweeps += count;
    }
    HIP_TRY(hipEventRecord(plan->ev1, stream));
    plan->last_sweeps = sweeps;
    plan->last_rebuilds = rebuilds;
    plan->timing_valid = true;

    a.gst = plan->d_gst;  // parity 0: every chunk has an even number of sweeps
    launch_finalize<T>(a, plan->grid, stream);
    launch_copy_out<T>(a, plan->grid, stream);
    HIP_TRY(hipGetLastError());

    plan->state_on_device = true;
    HIP_TRY(hipStreamSynchronize(stream));
    return read_state(plan, false);
}

}  // namespace

extern "C" {

emd_status emd_params_default(emd_params* p)
{
    if (!p) return fail(EMD_ERR_NULL_POINTER, "params is NULL");
    std::memset(p, 0, sizeof(*p));
    p->eps = 1e-4;
    p->xi = 0.5;
    p->zeta = 0.99;
    p->delta = 1e5;
    p->alpha1 = 0.0;
    p->alpha_max_factor = 1e6;
    p->tol_res = 1e-5;
    p->mass_tol = 1e-6;
    p->max_iter = 100000;
    p->check_every = 10;
    p->max_ls_trials = 40;
    p->ls_mode = EMD_LS_L2;
    p->mass_mode = EMD_MASS_BALANCE;
    p->precision = EMD_F32;
    p->sweeps_per_sync = 64;
    p->iters_per_sweep = 1;
    return EMD_SUCCESS;
}

emd_status emd_plan_create(const emd_gather_desc* h_desc, int32_t ngather, int64_t batch_len,
                           const emd_params* p, emd_plan** out)
{
    g_last_error.clear();
    if (!out) return fail(EMD_ERR_NULL_POINTER, "out is NULL");
    *out = nullptr;
    if (!h_desc) return fail(EMD_ERR_NULL_POINTER, "h_desc is NULL");
    if (ngather < 1) return fail(EMD_ERR_INVALID_ARGUMENT, "ngather must be >= 1");
    if (batch_len < 1) return fail(EMD_ERR_INVALID_ARGUMENT, "batch_len must be >= 1");
    emd_status st = validate_params(p);
    if (st != EMD_SUCCESS) return st;
    std::vector<std::pair<int64_t, int64_t>> spans;
    for (int g = 0; g < ngather; ++g) {
        const emd_gather_desc& d = h_desc[g];
        char msg[160];
        if (d.nr < 1 || d.nt < 1 || (int64_t)d.nr * d.nt > (int64_t)1 << 31) {
            std::snprintf(msg, sizeof msg, "gather %d: nr, nt must be >= 1 and nr*nt <= 2^31", g);
            return fail(EMD_ERR_INVALID_ARGUMENT, msg);
        }
        if (!(d.dx > 0.0) || !(d.dt > 0.0) || !std::isfinite(d.dx) || !std::isfinite(d.dt)) {
            std::snprintf(msg, sizeof msg, "gather %d: dx and dt must be finite and > 0", g);
            return fail(EMD_ERR_INVALID_ARGUMENT, msg);
        }
        // the sweep addresses a gather's padded field region with 32-bit byte offsets
        const int64_t region = (int64_t)d.nr * ((d.nt + 31) / 32 * 32) * (p->precision == EMD_F64 ? 8 : 4);
        if (region > ((int64_t)1 << 30)) {
            std::snprintf(msg, sizeof msg, "gather %d: nr * nt too large (at most 1 GiB per field)", g);
            return fail(EMD_ERR_INVALID_ARGUMENT, msg);
        }
        if (d.offset < 0 || d.offset + (int64_t)d.nr * d.nt > batch_len) {
            std::snprintf(msg, sizeof msg, "gather %d: [offset, offset + nr*nt) outside the batch", g);
            return fail(EMD_ERR_INVALID_ARGUMENT, msg);
        }
        spans.emplace_back(d.offset, d.offset + (int64_t)d.nr * d.nt);
    }
    std::sort(spans.begin(), spans.end());
    for (size_t k = 1; k < spans.size(); ++k)
        if (spans[k].first < spans[k - 1].second) return fail(EMD_ERR_INVALID_ARGUMENT, "gathers overlap");

    int dev = -1;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(EMD_ERR_DEVICE, "no HIP device");
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(EMD_ERR_DEVICE, std::string("this library is built for gfx950, device is ") + prop.gcnArchName);

    emd_plan* plan = new emd_plan();
    plan->device = dev;
    plan->ngather = ngather;
    plan->batch_len = batch_len;
    plan->params = *p;
    plan->desc.assign(h_desc, h_desc + ngather);
    plan->grows.assign(ngather, kDefaultRows);
    plan->elem = p->precision == EMD_F64 ? 8 : 4;
    plan->vec = p->precision == EMD_F64 ? 2 : 4;
    for (auto& d : plan->desc) plan->cells += (int64_t)d.nr * d.nt;
    auto cleanup = [&](emd_status s) {
        emd_plan_destroy(plan);
        return s;
    };
    st = build_tiles(plan);
    if (st != EMD_SUCCESS) return cleanup(st);
    const size_t fbytes = plan->elem * (size_t)plan->padded_len * 9;
    if (hipMalloc(&plan->d_fields, fbytes) != hipSuccess ||
        hipMalloc(&plan->d_gst, sizeof(GState) * 2 * ngather) != hipSuccess ||
        hipMalloc(&plan->d_done, sizeof(int32_t) * 64) != hipSuccess ||
        hipMalloc(&plan->d_adj, sizeof(double) * 4 * ngather) != hipSuccess ||
        hipMalloc(&plan->d_resume, sizeof(ResumeRec) * ngather) != hipSuccess) {
        std::string m = "cannot allocate the solver workspace (" + std::to_string(fbytes >> 20) + " MiB)";
        cleanup(EMD_SUCCESS);
        return fail(EMD_ERR_OUT_OF_MEMORY, m);
    }
    if (hipHostMalloc(&plan->h_done, sizeof(int32_t) * 16, hipHostMallocDefault) != hipSuccess) {
        cleanup(EMD_SUCCESS);
        return fail(EMD_ERR_OUT_OF_MEMORY, "cannot allocate pinned host memory");
    }
    if (hipMemset(plan->d_fields, 0, fbytes) != hipSuccess ||
        hipMemset(plan->d_gst, 0, sizeof(GState) * 2 * ngather) != hipSuccess ||
        hipMemset(plan->d_done, 0, sizeof(int32_t) * 64) != hipSuccess ||
        hipEventCreate(&plan->ev0) != hipSuccess || hipEventCreate(&plan->ev1) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        cleanup(EMD_SUCCESS);
        return fail(EMD_ERR_HIP, "workspace initialisation failed");
    }
    *out = plan;
    return EMD_SUCCESS;
}

emd_status emd_plan_destroy(emd_plan* plan)
{
    if (!plan) return EMD_SUCCESS;
    (void)hipDeviceSynchronize();
    destroy_graph(plan);
    if (plan->d_meta) (void)hipFree(plan->d_meta);
    if (plan->d_tiles) (void)hipFree(plan->d_tiles);
    if (plan->d_tiles_act) (void)hipFree(plan->d_tiles_act);
    if (plan->d_fields) (void)hipFree(plan->d_fields);
    if (plan->d_part) (void)hipFree(plan->d_part);
    if (plan->d_part_l1) (void)hipFree(plan->d_part_l1);
    if (plan->d_gst) (void)hipFree(plan->d_gst);
    if (plan->d_done) (void)hipFree(plan->d_done);
    if (plan->d_adj) (void)hipFree(plan->d_adj);
    if (plan->d_resume) (void)hipFree(plan->d_resume);
    if (plan->h_done) (void)hipHostFree(plan->h_done);
    if (plan->ev0) (void)hipEventDestroy(plan->ev0);
    if (plan->ev1) (void)hipEventDestroy(plan->ev1);
    delete plan;
    return EMD_SUCCESS;
}

emd_status emd_plan_set_params(emd_plan* plan, const emd_params* p)
{
    g_last_error.clear();
    if (!plan) return fail(EMD_ERR_NULL_POINTER, "plan is NULL");
    emd_status st = validate_params(p);
    if (st != EMD_SUCCESS) return st;
    if (p->precision != plan->params.precision)
        return fail(EMD_ERR_INVALID_ARGUMENT, "precision cannot change on an existing plan");
    st = check_device(plan);
    if (st != EMD_SUCCESS) return st;
    HIP_TRY(hipDeviceSynchronize());  // enqueued work may still read the gather table
    plan->params = *p;
    return build_tiles(plan);  // alpha_1 depends on delta and alpha1
}

emd_status emd_plan_set_tiling(emd_plan* plan, int32_t rows_per_tile)
{
    g_last_error.clear();
    if (!plan) return fail(EMD_ERR_NULL_POINTER, "plan is NULL");
    if (rows_per_tile < 0 || rows_per_tile > 1024)
        return fail(EMD_ERR_INVALID_ARGUMENT, "rows_per_tile must lie in [0, 1024]");
    emd_status st = check_device(plan);
    if (st != EMD_SUCCESS) return st;
    HIP_TRY(hipDeviceSynchronize());
    plan->rows = rows_per_tile == 0 ? kDefaultRows : rows_per_tile;
    plan->grows.assign(plan->ngather, plan->rows);
    return build_tiles(plan);
}

emd_status emd_plan_set_gather_tiling(emd_plan* plan, const int32_t* h_rows)
{
    g_last_error.clear();
    if (!plan || !h_rows) return fail(EMD_ERR_NULL_POINTER, "plan or h_rows is NULL");
    for (int g = 0; g < plan->ngather; ++g)
        if (h_rows[g] < 1 || h_rows[g] > 1024)
            return fail(EMD_ERR_INVALID_ARGUMENT, "rows per tile must lie in [1, 1024] (gather " +
                                                      std::to_string(g) + ")");
    emd_status st = check_device(plan);
    if (st != EMD_SUCCESS) return st;
    HIP_TRY(hipDeviceSynchronize());
    plan->grows.assign(h_rows, h_rows + plan->ngather);
    return build_tiles(plan);
}

emd_status emd_plan_set_history(emd_plan* plan, double* d_hist, int32_t capacity)
{
    g_last_error.clear();
    if (!plan) return fail(EMD_ERR_NULL_POINTER, "plan is NULL");
    if (d_hist && capacity < 1) return fail(EMD_ERR_INVALID_ARGUMENT, "capacity must be >= 1");
    if (!d_hist && capacity != 0) return fail(EMD_ERR_NULL_POINTER, "d_hist is NULL but capacity is not 0");
    emd_status st = check_device(plan);
    if (st != EMD_SUCCESS) return st;
    plan->d_hist = d_hist;
    plan->hist_cap = d_hist ? capacity : 0;
    return EMD_SUCCESS;
}

emd_status emd_plan_get_gather_tiling(const emd_plan* plan, int32_t* h_rows)
{
    g_last_error.clear();
    if (!plan || !h_rows) return fail(EMD_ERR_NULL_POINTER, "plan or h_rows is NULL");
    for (int g = 0; g < plan->ngather; ++g) h_rows[g] = plan->grows[g];
    return EMD_SUCCESS;
}

// Tile-height autotuner.  Gathers fall into 3 x 3 size buckets (tertiles of nt and
// of nr over the batch); bucket by bucket, largest first, each candidate height is
// tried for that bucket's gathers with the others fixed, keeping it when a short
// fixed-step solve of the whole batch (the production launch configuration: the
// captured chunk with its chains) runs faster by more than the timing noise.
emd_status emd_plan_autotune(emd_plan* plan, const void* s, int32_t sweeps, hipStream_t stream)
{
    g_last_error.clear();
    const Range range("emd_plan_autotune");
    if (!plan || !s) return fail(EMD_ERR_NULL_POINTER, "plan or s is NULL");
    if (sweeps == 0) sweeps = 48;
    if (sweeps < 4 || sweeps > 4096 || (sweeps & 1))
        return fail(EMD_ERR_INVALID_ARGUMENT, "sweeps must be even and lie in [4, 4096]");
    emd_status st = check_device(plan);
    if (st != EMD_SUCCESS) return st;
    const emd_params saved = plan->params;
    const std::vector<int> saved_rows = plan->grows;
    double* const saved_hist = plan->d_hist;
    plan->d_hist = nullptr;  // the timing solves record no residual history
    plan->params.ls_mode = EMD_LS_FIXED;
    plan->params.max_iter = sweeps - 2;  // max_iter + 2 sweeps: one captured chunk
    plan->params.check_every = sweeps - 2;
    plan->params.tol_res = 0.0;
    plan->params.sweeps_per_sync = sweeps;
    auto restore = [&](emd_status code) {
        plan->params = saved;
        plan->d_hist = saved_hist;
        if (code != EMD_SUCCESS) {
            const std::string msg = g_last_error;
            plan->grows = saved_rows;
            (void)build_tiles(plan);
            g_last_error = msg;
        }
        return code;
    };
    // one untimed solve captures the graph of this tiling; the fastest of the next
    // three is its time (one chunk is ~20 ms, where run-to-run noise is a few tenths
    // of a percent, as large as the differences between neighbouring heights)
    auto timed = [&](float& ms) -> emd_status {
        ms = 0.f;
        for (int r = 0; r < 4; ++r) {
            const emd_status e =
                plan->params.precision == EMD_F32
                    ? solve_impl<float>(plan, s, nullptr, nullptr, 0, nullptr, nullptr, 0, nullptr, nullptr, stream)
                    : solve_impl<double>(plan, s, nullptr, nullptr, 0, nullptr, nullptr, 0, nullptr, nullptr, stream);
            if (e != EMD_SUCCESS) return e;
            if (r == 0) continue;
            float t = 0.f;
            HIP_TRY(hipEventElapsedTime(&t, plan->ev0, plan->ev1));
            if (r == 1 || t < ms) ms = t;
        }
        return EMD_SUCCESS;
    };
    const int n = plan->ngather;
    std::vector<int> nts(n), nrs(n);
    for (int g = 0; g < n; ++g) {
        nts[g] = plan->desc[g].nt;
        nrs[g] = plan->desc[g].nr;
    }
    std::vector<int> snt = nts, snr = nrs;
    std::sort(snt.begin(), snt.end());
    std::sort(snr.begin(), snr.end());
    auto bin = [&](const std::vector<int>& sorted, int v) {
        return (v >= sorted[n / 3] ? 1 : 0) + (v >= sorted[(2 * n) / 3] ? 1 : 0);
    };
    std::vector<int> bucket(n);
    int64_t bcells[9] = {};
    for (int g = 0; g < n; ++g) {
        bucket[g] = 3 * bin(snt, nts[g]) + bin(snr, nrs[g]);
        bcells[bucket[g]] += (int64_t)nts[g] * nrs[g];
    }
    int order[9];
    for (int b = 0; b < 9; ++b) order[b] = b;
    std::stable_sort(order, order + 9, [&](int x, int y) { return bcells[x] > bcells[y]; });

    std::vector<int> best_rows = plan->grows;
    st = build_tiles(plan);
    if (st != EMD_SUCCESS) return restore(st);
    float best = 0.f;
    st = timed(best);
    if (st != EMD_SUCCESS) return restore(st);
    // Taller tiles than the default are not tried: at the end of a solve the last
    // gathers run alone and each launch lasts about one wave's march over its rows,
    // which a whole-batch timing does not see; whenever such timings chose 24 or 32
    // rows for a bucket, the full solve was slower.
    static const int kCand[] = {8, 12, kDefaultRows};
    for (int bi = 0; bi < 9; ++bi) {
        const int b = order[bi];
        if (bcells[b] == 0) continue;
        int cur = 0;
        for (int g = 0; g < n; ++g)
            if (bucket[g] == b) cur = best_rows[g];
        for (int c : kCand) {
            if (c == cur) continue;
            std::vector<int> trial = best_rows;
            for (int g = 0; g < n; ++g)
                if (bucket[g] == b) trial[g] = c;
            plan->grows = trial;
            st = build_tiles(plan);
            if (st != EMD_SUCCESS) return restore(st);
            float ms = 0.f;
            st = timed(ms);
            if (st != EMD_SUCCESS) return restore(st);
            if (ms < best * 0.997f) {
                best = ms;
                best_rows = trial;
            }
        }
    }
    plan->grows = best_rows;
    st = build_tiles(plan);
    return restore(st);
}

emd_status emd_plan_query(const emd_plan* plan, emd_plan_stats* out)
{
    g_last_error.clear();
    if (!plan || !out) return fail(EMD_ERR_NULL_POINTER, "plan or out is NULL");
    const emd_status rs = read_state(const_cast<emd_plan*>(plan), true);
    if (rs != EMD_SUCCESS) return rs;
    std::memset(out, 0, sizeof(*out));
    out->ngather = plan->ngather;
    out->tiles = plan->ntiles;
    out->rows_per_tile = plan->rows;
    out->samples_per_tile = OUT_LANES * plan->vec;
    out->batch_len = plan->batch_len;
    out->cells = plan->cells;
    out->workspace_bytes = plan->workspace_bytes;
    out->last_sweeps = plan->last_sweeps;
    out->last_cell_updates = plan->last_cell_updates;
    out->last_sweep_ms = 0.0;
    out->last_table_rebuilds = plan->last_rebuilds;
    if (plan->timing_valid) {
        float ms = 0.f;
        if (hipEventSynchronize(plan->ev1) == hipSuccess &&
            hipEventElapsedTime(&ms, plan->ev0, plan->ev1) == hipSuccess)
            out->last_sweep_ms = ms;
    }
    return EMD_SUCCESS;
}

emd_status emd_decompose(emd_plan* plan, const void* pcal, const void* pobs, void* s_out,
                         void* f_out, void* g_out, double* d_mass, hipStream_t stream)
{
    g_last_error.clear();
    const Range range("emd_decompose");
    if (!plan) return fail(EMD_ERR_NULL_POINTER, "plan is NULL");
    if (!pcal || !pobs || !s_out || !d_mass) return fail(EMD_ERR_NULL_POINTER, "pcal, pobs, s_out and d_mass are required");
    if (s_out == pcal || s_out == pobs) return fail(EMD_ERR_INVALID_ARGUMENT, "s_out aliases an input");
    emd_status st = check_device(plan);
    if (st != EMD_SUCCESS) return st;
    if (plan->params.precision == EMD_F32) {
        AuxArgs<float> a = aux_args<float>(plan);
        a.pcal = static_cast<const float*>(pcal);
        a.pobs = static_cast<const float*>(pobs);
        a.s_out = static_cast<float*>(s_out);
        a.f_out = static_cast<float*>(f_out);
        a.g_out = static_cast<float*>(g_out);
        a.mass_out = d_mass;
        launch_decompose<float>(a, plan->grid, stream);
    } else {
        AuxArgs<double> a = aux_args<double>(plan);
        a.pcal = static_cast<const double*>(pcal);
        a.pobs = static_cast<const double*>(pobs);
        a.s_out = static_cast<double*>(s_out);
        a.f_out = static_cast<double*>(f_out);
        a.g_out = static_cast<double*>(g_out);
        a.mass_out = d_mass;
        launch_decompose<double>(a, plan->grid, stream);
    }
    HIP_TRY(hipGetLastError());
    return EMD_SUCCESS;
}

emd_status emd_pdhg_solve(emd_plan* plan, const void* s, void* u, void* phi, int32_t warm_start,
                          const double* d_mass, double* d_emd, emd_solve_info* d_info,
                          hipStream_t stream)
{
    g_last_error.clear();
    const Range range("emd_pdhg_solve");
    if (!plan) return fail(EMD_ERR_NULL_POINTER, "plan is NULL");
    if (!s || !phi) return fail(EMD_ERR_NULL_POINTER, "s and phi are required");
    if (s == phi || s == u) return fail(EMD_ERR_INVALID_ARGUMENT, "s aliases an output");
    emd_status st = check_device(plan);
    if (st != EMD_SUCCESS) return st;
    if (plan->params.precision == EMD_F32)
        return solve_impl<float>(plan, s, u, phi, warm_start != 0, d_mass, nullptr, 0, d_emd, d_info, stream);
    return solve_impl<double>(plan, s, u, phi, warm_start != 0, d_mass, nullptr, 0, d_emd, d_info, stream);
}

emd_status emd_pdhg_solve_replay(emd_plan* plan, const void* s, void* u, void* phi,
                                 int32_t warm_start, const double* d_alpha, int32_t ld_alpha,
                                 double* d_emd, emd_solve_info* d_info, hipStream_t stream)
{
    g_last_error.clear();
    const Range range("emd_pdhg_solve_replay");
    if (!plan) return fail(EMD_ERR_NULL_POINTER, "plan is NULL");
    if (!s || !phi || !d_alpha) return fail(EMD_ERR_NULL_POINTER, "s, phi and d_alpha are required");
    if (s == phi || s == u) return fail(EMD_ERR_INVALID_ARGUMENT, "s aliases an output");
    if (ld_alpha < plan->params.max_iter)
        return fail(EMD_ERR_INVALID_ARGUMENT, "ld_alpha must be >= max_iter");
    emd_status st = check_device(plan);
    if (st != EMD_SUCCESS) return st;
    if (plan->params.precision == EMD_F32)
        return solve_impl<float>(plan, s, u, phi, warm_start != 0, nullptr, d_alpha, ld_alpha, d_emd, d_info, stream);
    return solve_impl<double>(plan, s, u, phi, warm_start != 0, nullptr, d_alpha, ld_alpha, d_emd, d_info, stream);
}

static_assert(sizeof(emd_gather_state) == sizeof(ResumeRec) &&
                  offsetof(emd_gather_state, iters) == offsetof(ResumeRec, iters) &&
                  offsetof(emd_gather_state, status) == offsetof(ResumeRec, status) &&
                  offsetof(emd_gather_state, rel_res) == offsetof(ResumeRec, rel_res) &&
                  offsetof(emd_gather_state, primal) == offsetof(ResumeRec, primal) &&
                  offsetof(emd_gather_state, transport) == offsetof(ResumeRec, transport),
              "emd_gather_state mirrors the resume record");

emd_status emd_solver_state(const emd_plan* plan, emd_gather_state* h_state)
{
    g_last_error.clear();
    if (!plan || !h_state) return fail(EMD_ERR_NULL_POINTER, "plan or h_state is NULL");
    const emd_status rs = read_state(const_cast<emd_plan*>(plan), true);
    if (rs != EMD_SUCCESS) return rs;
    if (plan->last_state.size() != (size_t)plan->ngather)
        return fail(EMD_ERR_INVALID_ARGUMENT, "the plan has not solved yet");
    for (int g = 0; g < plan->ngather; ++g) {
        const GState& s = plan->last_state[g];
        h_state[g].alpha = s.alpha;
        h_state[g].theta = s.theta;
        h_state[g].iters = s.iters;
        h_state[g].ls_trials = s.trials;
        h_state[g].status = s.status;
        h_state[g].pad = 0;
        h_state[g].rel_res = s.rel_res;
        h_state[g].primal = s.emd;
        h_state[g].transport = s.transport;
    }
    return EMD_SUCCESS;
}

emd_status emd_pdhg_solve_resume(emd_plan* plan, const void* s, void* u, void* phi,
                                 const emd_gather_state* h_state, const double* d_mass,
                                 double* d_emd, emd_solve_info* d_info, hipStream_t stream)
{
    g_last_error.clear();
    const Range range("emd_pdhg_solve_resume");
    if (!plan) return fail(EMD_ERR_NULL_POINTER, "plan is NULL");
    if (!s || !u || !phi || !h_state) return fail(EMD_ERR_NULL_POINTER, "s, u, phi and h_state are required");
    if (s == phi || s == u) return fail(EMD_ERR_INVALID_ARGUMENT, "s aliases an output");
    for (int g = 0; g < plan->ngather; ++g) {
        const emd_gather_state& r = h_state[g];
        const bool cont = r.status == EMD_GATHER_RUNNING || r.status == EMD_GATHER_MAX_ITER;
        if (r.status < EMD_GATHER_RUNNING || r.status > EMD_GATHER_MASS_IMBALANCE || r.iters < 0 ||
            r.ls_trials < 0 ||
            (cont && (!(r.alpha > 0.0) || !std::isfinite(r.alpha) || !std::isfinite(r.theta))))
            return fail(EMD_ERR_INVALID_ARGUMENT, "h_state[" + std::to_string(g) + "] is not a solver state");
    }
    emd_status st = check_device(plan);
    if (st != EMD_SUCCESS) return st;
    std::vector<ResumeRec> rec(plan->ngather);
    std::memcpy(rec.data(), h_state, sizeof(ResumeRec) * plan->ngather);
    if (plan->params.precision == EMD_F32)
        return solve_impl<float>(plan, s, u, phi, 1, d_mass, nullptr, 0, d_emd, d_info, stream, rec.data());
    return solve_impl<double>(plan, s, u, phi, 1, d_mass, nullptr, 0, d_emd, d_info, stream, rec.data());
}

emd_status emd_adjoint_source(emd_plan* plan, const void* phi, const void* pcal, const void* pobs,
                              const double* d_mass, const double* d_gbar, void* psi_out,
                              hipStream_t stream)
{
    g_last_error.clear();
    const Range range("emd_adjoint_source");
    if (!plan) return fail(EMD_ERR_NULL_POINTER, "plan is NULL");
    if (!phi || !psi_out) return fail(EMD_ERR_NULL_POINTER, "phi and psi_out are required");
    if (plan->params.mass_mode == EMD_MASS_UNIT && (!pcal || !pobs || !d_mass))
        return fail(EMD_ERR_NULL_POINTER, "unit mass mode needs pcal, pobs and d_mass");
    if (psi_out == phi || psi_out == pcal || psi_out == pobs)
        return fail(EMD_ERR_INVALID_ARGUMENT, "psi_out aliases an input");
    emd_status st = check_device(plan);
    if (st != EMD_SUCCESS) return st;
    if (plan->params.precision == EMD_F32) {
        AuxArgs<float> a = aux_args<float>(plan);
        a.phi_user = static_cast<const float*>(phi);
        a.pcal = static_cast<const float*>(pcal);
        a.pobs = static_cast<const float*>(pobs);
        a.mass = d_mass;
        a.gbar = d_gbar;
        a.psi_out = static_cast<float*>(psi_out);
        launch_adjoint<float>(a, plan->grid, stream);
    } else {
        AuxArgs<double> a = aux_args<double>(plan);
        a.phi_user = static_cast<const double*>(phi);
        a.pcal = static_cast<const double*>(pcal);
        a.pobs = static_cast<const double*>(pobs);
        a.mass = d_mass;
        a.gbar = d_gbar;
        a.psi_out = static_cast<double*>(psi_out);
        launch_adjoint<double>(a, plan->grid, stream);
    }
    HIP_TRY(hipGetLastError());
    return EMD_SUCCESS;
}

emd_status emd_lsd_misfit(emd_plan* plan, const void* pcal, const void* pobs, const double* d_gbar,
                          double* d_value, void* psi_out, hipStream_t stream)
{
    g_last_error.clear();
    const Range range("emd_lsd_misfit");
    if (!plan) return fail(EMD_ERR_NULL_POINTER, "plan is NULL");
    if (!pcal || !pobs || !d_value) return fail(EMD_ERR_NULL_POINTER, "pcal, pobs and d_value are required");
    if (psi_out && (psi_out == pcal || psi_out == pobs))
        return fail(EMD_ERR_INVALID_ARGUMENT, "psi_out aliases an input");
    emd_status st = check_device(plan);
    if (st != EMD_SUCCESS) return st;
    if (plan->params.precision == EMD_F32) {
        AuxArgs<float> a = aux_args<float>(plan);
        a.pcal = static_cast<const float*>(pcal);
        a.pobs = static_cast<const float*>(pobs);
        a.gbar = d_gbar;
        a.emd_out = d_value;
        a.psi_out = static_cast<float*>(psi_out);
        launch_lsd<float>(a, plan->grid, stream);
    } else {
        AuxArgs<double> a = aux_args<double>(plan);
        a.pcal = static_cast<const double*>(pcal);
        a.pobs = static_cast<const double*>(pobs);
        a.gbar = d_gbar;
        a.emd_out = d_value;
        a.psi_out = static_cast<double*>(psi_out);
        launch_lsd<double>(a, plan->grid, stream);
    }
    HIP_TRY(hipGetLastError());
    return EMD_SUCCESS;
}

}  // extern "C"

namespace {

// The two plans hold the same gathers, the coarse one grouped fr receivers by ft
// samples; returns the largest per-gather row count of the side the kernel walks.
emd_status check_transfer(const emd_plan* fine, const emd_plan* coarse, int32_t fr, int32_t ft,
                          bool walk_fine, int32_t& max_rows)
{
    if (!fine || !coarse) return fail(EMD_ERR_NULL_POINTER, "fine and coarse plans are required");
    if (fr < 1 || ft < 1) return fail(EMD_ERR_INVALID_ARGUMENT, "fr and ft must be >= 1");
    if (fine->ngather != coarse->ngather)
        return fail(EMD_ERR_INVALID_ARGUMENT, "the plans hold different numbers of gathers");
    if (fine->params.precision != coarse->params.precision)
        return fail(EMD_ERR_INVALID_ARGUMENT, "the plans have different precisions");
    if (fine->device != coarse->device) return fail(EMD_ERR_DEVICE, "the plans are on different devices");
    if (fine->ngather > 65535) return fail(EMD_ERR_UNSUPPORTED, "grid transfer takes at most 65535 gathers");
    max_rows = 0;
    for (int g = 0; g < fine->ngather; ++g) {
        const emd_gather_desc& f = fine->desc[g];
        const emd_gather_desc& c = coarse->desc[g];
        if (c.nr != (f.nr + fr - 1) / fr || c.nt != (f.nt + ft - 1) / ft)
            return fail(EMD_ERR_INVALID_ARGUMENT,
                        "gather " + std::to_string(g) + ": the coarse grid must be ceil(nr / fr) x ceil(nt / ft)");
        max_rows = std::max(max_rows, walk_fine ? f.nr : c.nr);
    }
    return check_device(const_cast<emd_plan*>(fine));
}

// one block per row of the walked grid, at most 2048 per gather (blocks then stride)
int transfer_blocks(int32_t rows) { return std::max(1, std::min(rows, 2048)); }

template <typename T>
XferArgs<T> xfer_args(const emd_plan* fine, const emd_plan* coarse, int32_t fr, int32_t ft)
{
    XferArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    a.meta_f = fine->d_meta;
    a.meta_c = coarse->d_meta;
    a.fr = fr;
    a.ft = ft;
    a.len_f = fine->batch_len;
    a.len_c = coarse->batch_len;
    return a;
}

}  // namespace

extern "C" {

emd_status emd_restrict(const emd_plan* fine, const emd_plan* coarse, int32_t fr, int32_t ft,
                        const void* fine_in, void* coarse_out, hipStream_t stream)
{
    g_last_error.clear();
    const Range range("emd_restrict");
    int32_t rows = 0;
    emd_status st = check_transfer(fine, coarse, fr, ft, false, rows);
    if (st != EMD_SUCCESS) return st;
    if (!fine_in || !coarse_out) return fail(EMD_ERR_NULL_POINTER, "fine_in and coarse_out are required");
    if (fine_in == coarse_out) return fail(EMD_ERR_INVALID_ARGUMENT, "coarse_out aliases fine_in");
    if (fine->params.precision == EMD_F32) {
        XferArgs<float> a = xfer_args<float>(fine, coarse, fr, ft);
        a.in = static_cast<const float*>(fine_in);
        a.out = static_cast<float*>(coarse_out);
        launch_restrict<float>(a, fine->ngather, transfer_blocks(rows), stream);
    } else {
        XferArgs<double> a = xfer_args<double>(fine, coarse, fr, ft);
        a.in = static_cast<const double*>(fine_in);
        a.out = static_cast<double*>(coarse_out);
        launch_restrict<double>(a, fine->ngather, transfer_blocks(rows), stream);
    }
    HIP_TRY(hipGetLastError());
    return EMD_SUCCESS;
}

emd_status emd_prolong(const emd_plan* coarse, const emd_plan* fine, int32_t fr, int32_t ft,
                       const void* u_c, const void* phi_c, void* u_f, void* phi_f, hipStream_t stream)
{
    g_last_error.clear();
    const Range range("emd_prolong");
    int32_t rows = 0;
    emd_status st = check_transfer(fine, coarse, fr, ft, true, rows);
    if (st != EMD_SUCCESS) return st;
    if (!u_f && !phi_f) return fail(EMD_ERR_NULL_POINTER, "u_f or phi_f is required");
    if ((u_f && !u_c) || (phi_f && !phi_c))
        return fail(EMD_ERR_NULL_POINTER, "each fine output needs its coarse input");
    if ((u_f && (u_f == u_c || u_f == phi_c)) || (phi_f && (phi_f == u_c || phi_f == phi_c)))
        return fail(EMD_ERR_INVALID_ARGUMENT, "a fine output aliases a coarse input");
    if (fine->params.precision == EMD_F32) {
        XferArgs<float> a = xfer_args<float>(fine, coarse, fr, ft);
        a.u_c = static_cast<const float*>(u_c);
        a.phi_c = static_cast<const float*>(phi_c);
        a.u_f = static_cast<float*>(u_f);
        a.phi_f = static_cast<float*>(phi_f);
        launch_prolong<float>(a, fine->ngather, transfer_blocks(rows), stream);
    } else {
        XferArgs<double> a = xfer_args<double>(fine, coarse, fr, ft);
        a.u_c = static_cast<const double*>(u_c);
        a.phi_c = static_cast<const double*>(phi_c);
        a.u_f = static_cast<double*>(u_f);
        a.phi_f = static_cast<double*>(phi_f);
        launch_prolong<double>(a, fine->ngather, transfer_blocks(rows), stream);
    }
    HIP_TRY(hipGetLastError());
    return EMD_SUCCESS;
}

}  // extern "C"

// ------------------------------------------------------------------ allocation-free decompose
//
// emd_decompose_noalloc keeps its per-gather partial sums in this file-scope device
// array instead of a plan's workspace: 64 gathers x 256 records x 3 doubles
// (384 KiB), which each device the library runs on holds until the process ends.
// Host code never passes the array's name to a kernel (in host code it stands for
// the array, not for its device address): the address comes from
// hipGetSymbolAddress, taken once per device with that device current, and that
// pointer is what the kernels receive.
namespace {

static_assert(kNdMaxGathers == EMD_NOALLOC_MAX_GATHERS, "the header states the scratch array's size");
__device__ __align__(256) double scratch[kNdMaxGathers * kNdBlocks * 3];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// The scratch array's address on the current device (found on the first call there),
// or NULL with the error set.
emd_status noalloc_scratch(double** out)
{
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(EMD_ERR_DEVICE, "device index beyond the supported 64");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        hipDeviceProp_t prop;
        HIP_TRY(hipGetDeviceProperties(&prop, dev));
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
            return fail(EMD_ERR_DEVICE, std::string("this library is built for gfx950, device is ") + prop.gcnArchName);
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(EMD_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return EMD_SUCCESS;
}

template <typename T>
void noalloc_launch(const emd_gather_desc* h_desc, int32_t ngather, int32_t mass_mode, const void* pcal,
                    const void* pobs, void* s_out, void* f_out, void* g_out, double* d_mass,
                    double* ws, hipStream_t stream)
{
    NdArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    a.ngather = ngather;
    a.mass_mode = mass_mode;
    for (int g = 0; g < ngather; ++g) {
        const emd_gather_desc& d = h_desc[g];
        a.g[g].off = d.offset;
        a.g[g].n = (int64_t)d.nr * d.nt;
        a.g[g].cm = (d.nr > 1 ? d.dx : 1.0) * (d.nt > 1 ? d.dt : 1.0);
    }
    a.pcal = static_cast<const T*>(pcal);
    a.pobs = static_cast<const T*>(pobs);
    a.s_out = static_cast<T*>(s_out);
    a.f_out = static_cast<T*>(f_out);
    a.g_out = static_cast<T*>(g_out);
    a.mass_out = d_mass;
    a.scratch = ws;
    launch_decompose_noalloc<T>(a, stream);
}

}  // namespace

extern "C" {

emd_status emd_decompose_noalloc(const emd_gather_desc* h_desc, int32_t ngather, int32_t precision,
                                 int32_t mass_mode, const void* pcal, const void* pobs, void* s_out,
                                 void* f_out, void* g_out, double* d_mass, hipStream_t stream)
{
    g_last_error.clear();
    const Range range("emd_decompose_noalloc");
    if (!h_desc) return fail(EMD_ERR_NULL_POINTER, "h_desc is NULL");
    if (!pcal || !pobs || !s_out || !d_mass) return fail(EMD_ERR_NULL_POINTER, "pcal, pobs, s_out and d_mass are required");
    if (s_out == pcal || s_out == pobs) return fail(EMD_ERR_INVALID_ARGUMENT, "s_out aliases an input");
    if (ngather < 1 || ngather > kNdMaxGathers)
        return fail(EMD_ERR_INVALID_ARGUMENT, "ngather must lie in [1, " + std::to_string(kNdMaxGathers) +
                                                  "] (the size of the library's static scratch array)");
    if (precision != EMD_F32 && precision != EMD_F64) return fail(EMD_ERR_INVALID_ARGUMENT, "unknown precision");
    if (mass_mode < EMD_MASS_BALANCE || mass_mode > EMD_MASS_NONE) return fail(EMD_ERR_INVALID_ARGUMENT, "unknown mass_mode");
    std::pair<int64_t, int64_t> spans[kNdMaxGathers];
    for (int g = 0; g < ngather; ++g) {
        const emd_gather_desc& d = h_desc[g];
        char msg[160];
        if (d.nr < 1 || d.nt < 1 || (int64_t)d.nr * d.nt > (int64_t)1 << 31) {
            std::snprintf(msg, sizeof msg, "gather %d: nr, nt must be >= 1 and nr*nt <= 2^31", g);
            return fail(EMD_ERR_INVALID_ARGUMENT, msg);
        }
        if (!(d.dx > 0.0) || !(d.dt > 0.0) || !std::isfinite(d.dx) || !std::isfinite(d.dt)) {
            std::snprintf(msg, sizeof msg, "gather %d: dx and dt must be finite and > 0", g);
            return fail(EMD_ERR_INVALID_ARGUMENT, msg);
        }
        if (d.offset < 0) {
            std::snprintf(msg, sizeof msg, "gather %d: offset must be >= 0", g);
            return fail(EMD_ERR_INVALID_ARGUMENT, msg);
        }
        spans[g] = {d.offset, d.offset + (int64_t)d.nr * d.nt};
    }
    std::sort(spans, spans + ngather);
    for (int k = 1; k < ngather; ++k)
        if (spans[k].first < spans[k - 1].second) return fail(EMD_ERR_INVALID_ARGUMENT, "gathers overlap");
    double* ws = nullptr;
    const emd_status st = noalloc_scratch(&ws);
    if (st != EMD_SUCCESS) return st;
    if (precision == EMD_F32)
        noalloc_launch<float>(h_desc, ngather, mass_mode, pcal, pobs, s_out, f_out, g_out, d_mass, ws, stream);
    else
        noalloc_launch<double>(h_desc, ngather, mass_mode, pcal, pobs, s_out, f_out, g_out, d_mass, ws, stream);
    HIP_TRY(hipGetLastError());
    return EMD_SUCCESS;
}

const char* emd_status_string(emd_status status)
{
    switch (status) {
    case EMD_SUCCESS: return "EMD_SUCCESS";
    case EMD_ERR_INVALID_ARGUMENT: return "EMD_ERR_INVALID_ARGUMENT";
    case EMD_ERR_NULL_POINTER: return "EMD_ERR_NULL_POINTER";
    case EMD_ERR_DEVICE: return "EMD_ERR_DEVICE";
    case EMD_ERR_HIP: return "EMD_ERR_HIP";
    case EMD_ERR_OUT_OF_MEMORY: return "EMD_ERR_OUT_OF_MEMORY";
    case EMD_ERR_UNSUPPORTED: return "EMD_ERR_UNSUPPORTED";
    default: return "EMD_ERR_UNKNOWN";
    }
}

const char* emd_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
