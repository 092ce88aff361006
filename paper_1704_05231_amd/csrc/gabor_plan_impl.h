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
    std::vector<int> adj_first;            // per frequency: its first adjoint job (O + 1 entries)
    int adj_max_kp = 0;
    int64_t adj_row_macs = 0, adj_col_macs = 0;
    AdjJob* d_ajobs = nullptr;
    void* d_adjW = nullptr;                // adjoint workspace (allocated, and grown, by adjoint calls)
    int64_t adj_cap = 0;                   // its bytes
    // recursive-smoother variant (gabor_bank_plan_iir)
    bool iir = false;
    int32_t n_ihj = 0, n_ivj = 0;
    int32_t iir_lc_h = 0, iir_lc_v = 0;    // longest chunk of each pass
    bool iir_reg_h = false, iir_reg_v = false;   // pass runs the register-resident kernel
    bool iir_rows_h = false;               // horizontal pass writes J rows (no transposed planes)
    IirJob* d_ihj = nullptr;
    IirJob* d_ivj = nullptr;
    float2* d_itw = nullptr;
    float* d_ifT = nullptr;
    float2* d_iJT = nullptr;
    float2* d_iJ = nullptr;
    float2* d_iscr = nullptr;
    int fused_op = FUSED_F32;
    bool use_ws = true;                    // wave-specialised kernel where built
    bool group_small = false;              // batch and apply: the small quarters in one launch
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
    // Replayable graphs of whole applies, keyed by their buffers and the
    // schedule (most recent last), captured on a plan-owned stream.
    struct ApplyGraph {
        const float* img;
        int64_t stride;
        void* out;
        std::vector<int> segs;             // the segment heights it was captured with
        gabor_batch batch;                 // the one-image batch it launches
        hipGraphExec_t exec;
    };
    std::vector<ApplyGraph> graphs;
    hipStream_t cap = nullptr;
    bool use_graphs = true;
    // per-kernel timing
    bool prof = false;
    struct Pending { int kind; hipEvent_t a, b; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> event_pool;
    std::vector<std::string> kind_names;
    std::vector<gabor_kernel_stat> stats;
};

namespace gabor {
// Drops the plan's cached apply graphs and the batches they replay.
void clear_apply_graphs(gabor_plan_s* p);
// Brackets one launch with events on its stream while the plan's profiling
// is on (gabor_profile_enable); the stat `name` holds one launch's
// algorithmic work.
struct LaunchTimer {
    gabor_plan p;
    hipStream_t s;
    int kind = -1;
    hipEvent_t a = nullptr, b = nullptr;
    LaunchTimer(gabor_plan plan, hipStream_t stream, const std::string& name, int64_t macs, int64_t bytes,
                bool enabled = true);
    ~LaunchTimer();
};
// Fused frequency i of the plan runs on the wave-specialised kernel.
inline bool fused_on_ws(const gabor_plan_s* p, int i)
{
    return p->launches[i].fused && p->use_ws && ws_supported(p->fused_op, p->launches[i].q);
}

// Two or more distinct small wave-specialised quarters: grouping them
// changes the launches of an apply.
inline bool has_small_group(const gabor_plan_s* p)
{
    int first = -1;
    for (int i = 0; i < p->O; ++i)
        if (fused_on_ws(p, i) && ws_small_quarter(p->fused_op, p->launches[i].q)) {
            if (first < 0) first = p->launches[i].q;
            else if (p->launches[i].q != first) return true;
        }
    return false;
}
// The plan's frequency table as the batch kernels read it (R, segment rows,
// scales, quarter per frequency).
std::vector<BatchFreq> batch_freq_table(const gabor_plan_s* p);
// Adjoint of the bank (gabor_plan.cpp).  Per frequency, the matrix-core
// kernel (fused frequencies of quarter <= 32: one partial plane per job) or
// the vector-ALU kernels (one partial plane); the planes lie on the image
// grid (zero boundary) or on the image extended by the frequency's R (mirror
// rule), and a last launch sums (or folds and sums) them into dL/df.  A
// zero-boundary plan with no matrix-core frequency runs the vector kernels
// once over every job, straight into dL/df.
struct AdjLayout {
    bool direct = false;
    std::vector<char> mfma;        // per frequency
    std::vector<int64_t> base;     // first float of its partial planes
    std::vector<int> planes;       // its partial planes
    std::vector<int64_t> jbase;    // first complex of its J planes (vector ALU)
    int64_t part_floats = 0;       // all partial planes
    int64_t j_offset = 0;          // bytes from an image's workspace to its J planes
    int64_t bytes = 0;             // workspace per image (a multiple of 256)
};
gabor_status adjoint_layout(const gabor_plan_s* p, AdjLayout* L);
// The launches for n_images images (G of image b at d_grad_out + b *
// g_bstride complex elements, its gradient at d_grad + b * grad_bstride) with
// a caller-provided workspace of at least n_images * L.bytes bytes; every
// byte of it that is read is first written by the same call.  `timed`
// brackets the launches with profiling events when profiling is on.
gabor_status adjoint_run(gabor_plan p, const AdjLayout& L, void* ws, const void* d_grad_out, int n_images,
                         int64_t g_bstride, float* d_grad, int64_t grad_bstride, int64_t grad_row_stride_elems,
                         hipStream_t stream, bool timed);
}  // namespace gabor

