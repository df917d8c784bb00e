// emd_launch.h -- kernel argument blocks and launch wrappers shared by the host
// code of the library and its kernel translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "emd_internal.h"

namespace emd {

template <typename T>
struct SweepArgs {
    const GatherMeta* meta;
    const Tile* tiles;
    int32_t ntiles, pad0;  // tiles in the table
    const T* s;            // padded source
    T* ux[2];
    T* ut[2];
    T* phi[2];
    T* R[2];
    double* part[2];       // [slots][NPART or NPART_L1] partial sums, by sweep parity
    GState* gst[2];        // [ngather], by sweep parity
    int32_t* done;         // gathers that have finished
    int32_t l1;            // 1: the l1 form of the linesearch test
    int32_t ips;           // fixed-step PDHG with 2 (k_sweep2) or 3 (k_sweep3) iterations
                           // per sweep; 0: one iteration per sweep (k_sweep)
    SolveScalars sc;
};

// Element-wise passes over the caller's batch layout and the padded workspace.
template <typename T>
struct AuxArgs {
    const GatherMeta* meta;
    const Tile* tiles;
    int32_t ntiles, pad0, ngather, mass_mode;
    double mass_tol;
    // caller's buffers (dense [nr][nt] at meta.uoff)
    const T* pcal;
    const T* pobs;
    const T* s_user;
    T* s_out;
    T* f_out;
    T* g_out;
    const T* u_user_in;   // warm start [u^x | u^t] or NULL
    const T* phi_user_in; // warm start or NULL
    T* u_user_out;        // NULL: not returned
    T* phi_user_out;
    T* psi_out;
    const T* phi_user;    // adjoint input
    int64_t batch_len;
    const double* mass;   // [ngather][3]
    double* mass_out;     // [ngather][3]
    const double* gbar;   // [ngather] or NULL
    double* adj;          // [ngather][4] adjoint scalars
    // workspace
    T* s_pad;
    T* ux[2];
    T* ut[2];
    T* phi[2];
    T* R[2];
    double* part;         // [tiles][NPART]
    GState* gst;          // parity-0 state (initial / final)
    int32_t* done;
    double* emd_out;      // [ngather] or NULL
    void* info_out;       // emd_solve_info[ngather] or NULL
    const ResumeRec* resume;  // [ngather]: continue from a checkpoint, or NULL
    double eps, delta_unused, alpha_max_factor;
};

// Grid transfer between a fine plan and a coarse plan of the same gathers, grouped
// fr receivers by ft samples (caller's batch layout on both sides).
template <typename T>
struct XferArgs {
    const GatherMeta* meta_f;  // fine plan's gathers
    const GatherMeta* meta_c;  // coarse plan's gathers (same order)
    int32_t fr, ft;
    int64_t len_f, len_c;      // batch lengths (offset of u^t after u^x)
    const T* in;               // restriction: fine field
    T* out;                    // restriction: coarse field
    const T* u_c;              // prolongation: coarse [u^x | u^t] or NULL
    const T* phi_c;            //   coarse phi or NULL
    T* u_f;                    //   fine [u^x | u^t] or NULL
    T* phi_f;                  //   fine phi or NULL
};

// The plan-free decompose: gathers described in the kernel arguments (at most
// kNdMaxGathers), per-gather partial sums in a caller-provided scratch array of
// kNdMaxGathers * kNdBlocks * 3 doubles.
constexpr int kNdMaxGathers = 64;
constexpr int kNdBlocks = 256;  // partial-sum records per gather (one per block)

struct NdGather {
    int64_t off;  // element offset in the caller's batch buffers
    int64_t n;    // nr * nt
    double cm;    // cell measure
};

template <typename T>
struct NdArgs {
    int32_t ngather, mass_mode;
    NdGather g[kNdMaxGathers];
    const T* pcal;
    const T* pobs;
    T* s_out;
    T* f_out;
    T* g_out;
    double* mass_out;  // [ngather][3]
    double* scratch;   // [kNdMaxGathers][kNdBlocks][3]
};

template <typename T> void launch_decompose_noalloc(const NdArgs<T>& a, hipStream_t stream);

template <typename T> void launch_sweep(const SweepArgs<T>& a, int parity, int grid, hipStream_t stream);
template <typename T> void launch_restrict(const XferArgs<T>& a, int ngather, int blocks, hipStream_t stream);
template <typename T> void launch_prolong(const XferArgs<T>& a, int ngather, int blocks, hipStream_t stream);
template <typename T> void launch_copy_in(const AuxArgs<T>& a, int warm, int grid, hipStream_t stream);
template <typename T> void launch_gather_init(const AuxArgs<T>& a, hipStream_t stream);
template <typename T> void launch_copy_out(const AuxArgs<T>& a, int grid, hipStream_t stream);
template <typename T> void launch_finalize(const AuxArgs<T>& a, int grid, hipStream_t stream);
template <typename T> void launch_decompose(const AuxArgs<T>& a, int grid, hipStream_t stream);
template <typename T> void launch_adjoint(const AuxArgs<T>& a, int grid, hipStream_t stream);
template <typename T> void launch_lsd(const AuxArgs<T>& a, int grid, hipStream_t stream);
void launch_zero_counter(int32_t* counter, hipStream_t stream);

}  // namespace emd
