// libgabor host side: argument validation, the bank plan of Algorithm 1
// (Sec. II-B) and the C ABI declared in include/libgabor.h.
//
// The plan turns (Omega, Sigma, Theta) into
//   - per frequency: the radius R and the reversed, zero-padded tap tables of
//     the horizontal and vertical 1-D passes, computed in FP64 and rounded to
//     FP32 once;
//   - horizontal passes: one per orientation that is not the pi - theta
//     partner of an earlier one (Eq. (13): J_(pi-theta) = conj(J_theta));
//   - vertical jobs: one per horizontal result, producing theta and, when
//     present, its partner pi - theta from the same J (Eq. (15)-(16)).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/libgabor.h"
#include "gabor_internal.h"

using namespace gabor;

struct gabor_plan_s {
    int32_t H = 0, W = 0, O = 0, N = 0;
    int32_t boundary = 0;
    int32_t precision = 0;
    std::vector<FreqDesc> freqs;
    std::vector<RowGroup> row_groups;
    std::vector<int32_t> job_first, job_count;   // per frequency, into jobs
    std::vector<ColJob> jobs;
    int32_t n_planes = 0;
    int32_t n_row_passes = 0, n_col_passes = 0;
    int64_t row_macs = 0, col_macs = 0;
    int64_t workspace_bytes = 0;
    float* d_taps = nullptr;
    ColJob* d_jobs = nullptr;
    float2* d_J = nullptr;
    // per-kernel timing
    bool prof = false;
    struct Pending { int kind; hipEvent_t a, b; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> event_pool;
    std::vector<std::string> kind_names;
    std::vector<gabor_kernel_stat> stats;
};

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kPairTol = 1e-12;
constexpr int kMaxRadius = 255;

bool env_flag(const char* name)
{
    const char* v = std::getenv(name);
    return v && *v && std::strcmp(v, "0") != 0;
}

// cos/sin of theta, exact at multiples of pi/2 so that theta = 0 and
// theta = pi/2 take the real-J / real-tap paths (the paper's N_h orientation
// k = N/2 has w cos(theta) = 0 exactly).
void exact_cos_sin(double th, double* c, double* s)
{
    const double q = th / (0.5 * kPi);
    const double r = std::nearbyint(q);
    if (std::fabs(q - r) < kPairTol) {
        long long k = ((long long)r % 4 + 4) % 4;
        static const double tc[4] = {1.0, 0.0, -1.0, 0.0}, ts[4] = {0.0, 1.0, 0.0, -1.0};
        *c = tc[k];
        *s = ts[k];
    } else {
        *c = std::cos(th);
        *s = std::sin(th);
    }
}

void release(gabor_plan p)
{
    if (!p) return;
    for (auto& q : p->pending) { (void)hipEventDestroy(q.a); (void)hipEventDestroy(q.b); }
    for (hipEvent_t e : p->event_pool) (void)hipEventDestroy(e);
    if (p->d_taps) (void)hipFree(p->d_taps);
    if (p->d_jobs) (void)hipFree(p->d_jobs);
    if (p->d_J) (void)hipFree(p->d_J);
    delete p;
}

hipEvent_t take_event(gabor_plan p)
{
    if (!p->event_pool.empty()) {
        hipEvent_t e = p->event_pool.back();
        p->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

int kind_index(gabor_plan p, const char* name)
{
    for (size_t i = 0; i < p->kind_names.size(); ++i)
        if (p->kind_names[i] == name) return (int)i;
    p->kind_names.push_back(name);
    gabor_kernel_stat st{};
    std::strncpy(st.name, name, sizeof(st.name) - 1);
    p->stats.push_back(st);
    return (int)p->kind_names.size() - 1;
}

// Brackets one launch with events when profiling is on.
struct LaunchTimer {
    gabor_plan p;
    hipStream_t s;
    int kind = -1;
    hipEvent_t a = nullptr, b = nullptr;
    LaunchTimer(gabor_plan plan, hipStream_t stream, const char* name) : p(plan), s(stream)
    {
        if (!p->prof) return;
        kind = kind_index(p, name);
        a = take_event(p);
        b = take_event(p);
        if (a && b && hipEventRecord(a, s) == hipSuccess) return;
        if (a) p->event_pool.push_back(a);
        if (b) p->event_pool.push_back(b);
        a = b = nullptr;
    }
    ~LaunchTimer()
    {
        if (!a) return;
        if (hipEventRecord(b, s) == hipSuccess) p->pending.push_back({kind, a, b});
        else { p->event_pool.push_back(a); p->event_pool.push_back(b); }
    }
};

struct RowPass {
    double wc;      // w cos(theta)
    bool real;      // wc == 0: J is real
    int32_t job;    // index of the vertical job consuming it
};

}  // namespace

extern "C" const char* gabor_status_string(gabor_status s)
{
    switch (s) {
        case GABOR_OK: return "GABOR_OK";
        case GABOR_ERR_INVALID_ARG: return "GABOR_ERR_INVALID_ARG";
        case GABOR_ERR_OUT_OF_MEMORY: return "GABOR_ERR_OUT_OF_MEMORY";
        case GABOR_ERR_DEVICE: return "GABOR_ERR_DEVICE";
        case GABOR_ERR_UNSUPPORTED: return "GABOR_ERR_UNSUPPORTED";
    }
    return "GABOR_ERR_UNKNOWN";
}

extern "C" gabor_status gabor_bank_plan(gabor_plan* out, int32_t height, int32_t width,
                                        int32_t n_freq, const double* omega, const double* sigma,
                                        int32_t n_orient, const double* theta,
                                        double radius_sigmas, gabor_boundary boundary,
                                        gabor_precision precision, void* hip_stream)
{
    if (!out) return GABOR_ERR_INVALID_ARG;
    *out = nullptr;
    if (height <= 0 || width <= 0 || n_freq <= 0 || n_orient <= 0) return GABOR_ERR_INVALID_ARG;
    if (!omega || !sigma) return GABOR_ERR_INVALID_ARG;
    if (!std::isfinite(radius_sigmas) || radius_sigmas < 0.0) return GABOR_ERR_INVALID_ARG;
    if (boundary != GABOR_BOUNDARY_ZERO && boundary != GABOR_BOUNDARY_MIRROR) return GABOR_ERR_INVALID_ARG;
    if ((int)precision < (int)GABOR_PREC_FP32 || (int)precision > (int)GABOR_PREC_FP16)
        return GABOR_ERR_INVALID_ARG;
    for (int i = 0; i < n_freq; ++i)
        if (!std::isfinite(omega[i]) || !std::isfinite(sigma[i]) || !(sigma[i] > 0.0))
            return GABOR_ERR_INVALID_ARG;
    if (theta)
        for (int k = 0; k < n_orient; ++k)
            if (!std::isfinite(theta[k])) return GABOR_ERR_INVALID_ARG;
    // Limits of this build: in-plane indices are 32-bit, one grid row per
    // image row, and the vertical pass stages (64 + Kp) J rows of a 32-column
    // tile in LDS (<= 160 KiB on gfx950), which bounds R at 255.
    if ((int64_t)height * width > (int64_t)INT32_MAX || height > 65535) return GABOR_ERR_UNSUPPORTED;
    for (int i = 0; i < n_freq; ++i)
        if (std::floor(radius_sigmas * sigma[i] + 0.5) > (double)kMaxRadius) return GABOR_ERR_UNSUPPORTED;
    if (precision != GABOR_PREC_FP32) return GABOR_ERR_UNSUPPORTED;

    gabor_plan p = new (std::nothrow) gabor_plan_s;
    if (!p) return GABOR_ERR_OUT_OF_MEMORY;
    p->H = height;
    p->W = width;
    p->O = n_freq;
    p->N = n_orient;
    p->boundary = boundary;
    p->precision = precision;

    // Orientation geometry, shared by every frequency.
    std::vector<double> cs(n_orient), sn(n_orient);
    for (int k = 0; k < n_orient; ++k) {
        const double th = theta ? theta[k] : kPi * (double)k / (double)n_orient;
        exact_cos_sin(th, &cs[k], &sn[k]);
    }

    std::vector<float> taps;
    const int64_t npix = (int64_t)height * width;
    for (int i = 0; i < n_freq; ++i) {
        FreqDesc fd;
        fd.R = (int)std::floor(radius_sigmas * sigma[i] + 0.5);
        fd.K = 2 * fd.R + 1;
        fd.Kp = (fd.K + kTapBlock - 1) / kTapBlock * kTapBlock;
        p->freqs.push_back(fd);
        // S(t), unit sum over |t| <= R.
        std::vector<double> S(fd.K);
        double sum = 0.0;
        for (int t = -fd.R; t <= fd.R; ++t) {
            S[t + fd.R] = std::exp(-(double)t * t / (2.0 * sigma[i] * sigma[i]));
            sum += S[t + fd.R];
        }
        for (double& v : S) v /= sum;

        // Pair orientations (Eq. (13)-(16)) and create the vertical jobs.
        std::vector<char> used(n_orient, 0);
        std::vector<RowPass> cplx, real;
        const int job0 = (int)p->jobs.size();
        for (int n = 0; n < n_orient; ++n) {
            if (used[n]) continue;
            used[n] = 1;
            ColJob jb{};
            jb.freq = i;
            jb.out_a = i * n_orient + n;
            jb.out_b = -1;
            const double wc = omega[i] * cs[n], ws = omega[i] * sn[n];
            jb.j_real = (wc == 0.0);
            jb.c_real = (ws == 0.0);
            if (!jb.j_real) {
                for (int m = n + 1; m < n_orient; ++m)
                    if (!used[m] && std::fabs(cs[m] + cs[n]) < kPairTol && std::fabs(sn[m] - sn[n]) < kPairTol) {
                        jb.out_b = i * n_orient + m;
                        used[m] = 1;
                        break;
                    }
            }
            // Column taps (reversed): c(R - T), d(R - T) with k(t) = S(t) e^{i ws t}.
            jb.tap_off = (int)taps.size();
            for (int T = 0; T < fd.Kp; ++T) {
                const int t = fd.R - T;
                const double s = T < fd.K ? S[T] : 0.0;   // S is symmetric: S(R-T) = S[T]
                taps.push_back((float)(s * std::cos(ws * t)));
                taps.push_back((float)(s * std::sin(ws * t)));
            }
            const int convs = (jb.c_real ? 1 : 2) * (jb.j_real ? 1 : 2);
            p->col_macs += (int64_t)convs * fd.K * npix;
            p->n_col_passes += 1;
            (jb.j_real ? real : cplx).push_back(RowPass{wc, (bool)jb.j_real, (int)p->jobs.size()});
            p->jobs.push_back(jb);
        }
        p->job_first.push_back(job0);
        p->job_count.push_back((int)p->jobs.size() - job0);

        // Horizontal groups: up to 6 complex passes plus at most one real pass
        // share one staged image row.
        size_t ci = 0, ri = 0;
        while (ci < cplx.size() || ri < real.size()) {
            RowGroup g{};
            g.freq = i;
            g.n_cplx = (int)std::min<size_t>(6, cplx.size() - ci);
            g.n_real = ri < real.size() ? 1 : 0;
            g.plane0 = p->n_planes;
            g.tap_off = (int)taps.size();
            const int NT = 2 * g.n_cplx + g.n_real;
            std::vector<const RowPass*> members;
            for (int c = 0; c < g.n_cplx; ++c) members.push_back(&cplx[ci + c]);
            if (g.n_real) members.push_back(&real[ri]);
            for (int T = 0; T < fd.Kp; ++T) {
                const int t = fd.R - T;
                const double s = T < fd.K ? S[T] : 0.0;
                for (int c = 0; c < g.n_cplx; ++c) {
                    taps.push_back((float)(s * std::cos(members[c]->wc * t)));
                    taps.push_back((float)(s * std::sin(members[c]->wc * t)));
                }
                if (g.n_real) taps.push_back((float)s);
            }
            (void)NT;
            for (size_t m = 0; m < members.size(); ++m) {
                p->jobs[members[m]->job].plane = g.plane0 + (int)m;
                const int convs = members[m]->real ? 1 : 2;
                p->row_macs += (int64_t)convs * fd.K * npix;
                p->n_row_passes += 1;
            }
            p->n_planes += (int)members.size();
            p->row_groups.push_back(g);
            ci += g.n_cplx;
            ri += g.n_real;
        }
    }

    // Device tables and workspace.
    const size_t taps_bytes = taps.size() * sizeof(float);
    const size_t jobs_bytes = p->jobs.size() * sizeof(ColJob);
    const size_t J_bytes = (size_t)p->n_planes * (size_t)npix * sizeof(float2);
    p->workspace_bytes = (int64_t)(taps_bytes + jobs_bytes + J_bytes);
    if (env_flag("LIBGABOR_FAIL_ALLOC")) {
        release(p);
        return GABOR_ERR_OUT_OF_MEMORY;
    }
    hipStream_t stream = (hipStream_t)hip_stream;
    hipError_t e;
    if ((e = hipMalloc((void**)&p->d_taps, taps_bytes)) != hipSuccess ||
        (e = hipMalloc((void**)&p->d_jobs, jobs_bytes)) != hipSuccess ||
        (e = hipMalloc((void**)&p->d_J, J_bytes)) != hipSuccess) {
        release(p);
        return e == hipErrorOutOfMemory ? GABOR_ERR_OUT_OF_MEMORY : GABOR_ERR_DEVICE;
    }
    if (hipMemcpyAsync(p->d_taps, taps.data(), taps_bytes, hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipMemcpyAsync(p->d_jobs, p->jobs.data(), jobs_bytes, hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess) {
        release(p);
        return GABOR_ERR_DEVICE;
    }
    *out = p;
    return GABOR_OK;
}

extern "C" gabor_status gabor_bank_apply(gabor_plan p, const float* d_image, int64_t row_stride_elems,
                                         void* d_out, void* hip_stream)
{
    if (!p || !d_image || !d_out) return GABOR_ERR_INVALID_ARG;
    if (row_stride_elems < p->W) return GABOR_ERR_INVALID_ARG;
    hipStream_t stream = (hipStream_t)hip_stream;
    for (const RowGroup& g : p->row_groups) {
        LaunchTimer tm(p, stream, "row_fp32");
        if (launch_row_fp32(d_image, row_stride_elems, p->H, p->W, p->boundary, p->freqs[g.freq], g,
                            p->d_taps, p->d_J, stream) != hipSuccess)
            return GABOR_ERR_DEVICE;
    }
    for (int i = 0; i < p->O; ++i) {
        LaunchTimer tm(p, stream, "col_fp32");
        if (launch_col_fp32(p->d_J, p->H, p->W, p->boundary, p->freqs[i], p->d_jobs + p->job_first[i],
                            p->job_count[i], p->d_taps, (float2*)d_out, stream) != hipSuccess)
            return GABOR_ERR_DEVICE;
    }
    return GABOR_OK;
}

extern "C" gabor_status gabor_bank_destroy(gabor_plan p)
{
    release(p);
    return GABOR_OK;
}

extern "C" gabor_status gabor_profile_enable(gabor_plan p, int32_t enable)
{
    if (!p) return GABOR_ERR_INVALID_ARG;
    for (auto& q : p->pending) {
        (void)hipEventSynchronize(q.b);
        p->event_pool.push_back(q.a);
        p->event_pool.push_back(q.b);
    }
    p->pending.clear();
    for (auto& st : p->stats) { st.launches = 0; st.total_ms = 0.0; }
    p->prof = enable != 0;
    return GABOR_OK;
}

extern "C" gabor_status gabor_profile_read(gabor_plan p, gabor_kernel_stat* stats, int32_t capacity,
                                           int32_t* n_stats)
{
    if (!p || !n_stats || capacity < 0 || (capacity > 0 && !stats)) return GABOR_ERR_INVALID_ARG;
    gabor_status rc = GABOR_OK;
    for (auto& q : p->pending) {
        float ms = 0.0f;
        if (hipEventSynchronize(q.b) != hipSuccess || hipEventElapsedTime(&ms, q.a, q.b) != hipSuccess)
            rc = GABOR_ERR_DEVICE;
        else {
            p->stats[q.kind].launches += 1;
            p->stats[q.kind].total_ms += ms;
        }
        p->event_pool.push_back(q.a);
        p->event_pool.push_back(q.b);
    }
    p->pending.clear();
    *n_stats = (int32_t)p->stats.size();
    for (int32_t i = 0; i < capacity && i < (int32_t)p->stats.size(); ++i) stats[i] = p->stats[i];
    return rc;
}

extern "C" gabor_status gabor_bank_plan_info(gabor_plan p, gabor_plan_info* info)
{
    if (!p || !info) return GABOR_ERR_INVALID_ARG;
    info->height = p->H;
    info->width = p->W;
    info->n_freq = p->O;
    info->n_orient = p->N;
    int mr = 0;
    for (const FreqDesc& f : p->freqs) mr = std::max(mr, f.R);
    info->max_radius = mr;
    info->n_row_passes = p->n_row_passes;
    info->n_col_passes = p->n_col_passes;
    info->precision = p->precision;
    info->workspace_bytes = p->workspace_bytes;
    info->real_macs = p->row_macs + p->col_macs;
    info->row_real_macs = p->row_macs;
    info->col_real_macs = p->col_macs;
    return GABOR_OK;
}
