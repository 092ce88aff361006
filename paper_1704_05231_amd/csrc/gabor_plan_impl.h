// Private definition of the bank plan, shared by the plan, apply and batch
// host code.  Not part of the public C ABI.
#pragma once

#include <string>
#include <vector>

#include "../../include/libgabor.h"
#include "gabor_internal.h"

namespace gabor {
// How one frequency is computed: the fused kernel (jobs in fjobs) or the
// two-pass kernels (jobs in jobs, J planes written by the row groups).
struct FreqLaunch {
    bool fused;
    int q;            // operand quarter: contracted length 4q (fused)
    int seg_rows;     // strip segment rows (fused)
    float in_scale, mid_scale, out_scale, tap_scale[2];
    int first;        // first job
    int count;        // jobs
    int64_t macs;     // algorithmic real MACs of the launch (vertical, plus horizontal when fused)
    int64_t bytes;    // algorithmic bytes of the launch
};
const char* const kFusedNames[5] = {"stream_f32", "stream_bf16", "stream_bf16x3", "stream_f16", "stream_f16x3"};
const char* const kWsNames[5] = {"ws_f32", "ws_bf16", "ws_bf16x3", "ws_f16", "ws_f16x3"};
enum { ALGO_AUTO = 0, ALGO_TWOPASS = 1 };
}  // namespace gabor

using namespace gabor;

struct gabor_plan_s {
    int32_t H = 0, W = 0, O = 0, N = 0;
    int32_t boundary = 0;
    int32_t precision = 0;
    std::vector<FreqDesc> freqs;
    std::vector<RowGroup> row_groups;
    std::vector<int64_t> row_group_macs;       // per row group
    std::vector<ColJob> jobs;              // two-pass vertical jobs
    std::vector<FusedJob> fjobs;           // fused jobs
    std::vector<FreqLaunch> launches;      // per frequency
    std::vector<int> order;                // launch order of the frequencies
    std::vector<AdjJob> ajobs;             // adjoint jobs (every horizontal result)
    int adj_max_kp = 0;
    int64_t adj_row_macs = 0, adj_col_macs = 0;
    AdjJob* d_ajobs = nullptr;
    float2* d_adjJ = nullptr;              // adjoint workspace, allocated by the first adjoint call
    float* d_adjP = nullptr;   // matrix-core adjoint: one partial plane per job (at first use)
    // recursive-smoother variant (gabor_bank_plan_iir)
    bool iir = false;
    int32_t n_ihj = 0, n_ivj = 0;
    IirJob* d_ihj = nullptr;
    IirJob* d_ivj = nullptr;
    float2* d_itw = nullptr;
    float* d_ifT = nullptr;
    float2* d_iJT = nullptr;
    float2* d_iJ = nullptr;
    float2* d_iscr = nullptr;
    int fused_op = FUSED_F32;
    bool use_ws = true;                    // wave-specialised kernel where built
    int32_t n_planes = 0;
    int32_t n_row_passes = 0, n_col_passes = 0;
    int64_t row_macs = 0, col_macs = 0;
    int64_t workspace_bytes = 0;
    float* d_taps = nullptr;
    ColJob* d_jobs = nullptr;
    FusedJob* d_fjobs = nullptr;
    float2* d_J = nullptr;
    // Fork/join of the per-frequency launches: auxiliary streams (default
    // priority) joined back to the caller's stream with events.
    std::vector<hipStream_t> aux;
    std::vector<hipEvent_t> fork_ev, join_ev;
    // per-kernel timing
    bool prof = false;
    struct Pending { int kind; hipEvent_t a, b; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> event_pool;
    std::vector<std::string> kind_names;
    std::vector<gabor_kernel_stat> stats;
};

namespace gabor {
// Fused frequency i of the plan runs on the wave-specialised kernel.
inline bool fused_on_ws(const gabor_plan_s* p, int i)
{
    return p->launches[i].fused && p->use_ws && ws_supported(p->fused_op, p->launches[i].q);
}
// The plan's frequency table as the batch kernels read it (R, segment rows,
// scales, quarter per frequency).
std::vector<BatchFreq> batch_freq_table(const gabor_plan_s* p);
// Adjoint of the bank (gabor_plan.cpp): which kernels a plan's adjoint runs
// (mfma: the matrix-core kernels) and the workspace bytes they need; then
// the launches with a caller-provided workspace of at least that size.
gabor_status adjoint_workspace(gabor_plan p, bool* mfma, int64_t* bytes);
gabor_status adjoint_run(gabor_plan p, bool mfma, void* ws, const void* d_grad_out, float* d_grad_image,
                         int64_t grad_row_stride_elems, hipStream_t stream, bool timed);
}  // namespace gabor

