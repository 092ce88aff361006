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
#include <array>
#include <complex>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/libgabor.h"
#include "gabor_internal.h"

using namespace gabor;

#include "gabor_plan_impl.h"

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
    if (p->d_fjobs) (void)hipFree(p->d_fjobs);
    if (p->d_J) (void)hipFree(p->d_J);
    if (p->d_ajobs) (void)hipFree(p->d_ajobs);
    if (p->d_adjW) (void)hipFree(p->d_adjW);
    for (void* q : {(void*)p->d_ihj, (void*)p->d_ivj, (void*)p->d_itw, (void*)p->d_ifT, (void*)p->d_iJT,
                    (void*)p->d_iJ, (void*)p->d_iscr})
        if (q) (void)hipFree(q);
    clear_apply_graphs(p);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    for (hipStream_t st : p->aux) (void)hipStreamDestroy(st);
    for (hipEvent_t e : p->fork_ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : p->join_ev) (void)hipEventDestroy(e);
    delete p;
}

struct RowPass {
    double wc;      // w cos(theta)
    bool real;      // wc == 0: J is real
    int32_t job;    // index of the vertical job consuming it
};


// One fused-kernel launch: all jobs of frequency i over the whole image,
// strip segments of seg_rows rows.
hipError_t launch_fused_freq(gabor_plan p, int i, const float* d_image, int64_t stride, void* d_out,
                             int seg_rows, hipStream_t s, int n_images = 1, int64_t img_bstride = 0,
                             int64_t out_bstride = 0)
{
    const FreqLaunch& fl = p->launches[i];
    StreamArgs sa{};
    sa.img = d_image;
    sa.stride = stride;
    sa.H = p->H;
    sa.W = p->W;
    sa.boundary = p->boundary;
    sa.R = p->freqs[i].R;
    sa.seg_rows = seg_rows;
    sa.n_xs = (p->W + stream_strip_width() - 1) / stream_strip_width();
    sa.n_ys = (p->H + seg_rows - 1) / seg_rows;
    sa.n_jobs = fl.count;
    sa.jobs = p->d_fjobs + fl.first;
    sa.taps = p->d_taps;
    sa.out = (float2*)d_out;
    sa.in_scale = fl.in_scale;
    sa.mid_scale = fl.mid_scale;
    sa.out_scale = fl.out_scale;
    sa.tap_scale[0] = fl.tap_scale[0];
    sa.tap_scale[1] = fl.tap_scale[1];
    sa.n_images = n_images;
    sa.img_bstride = img_bstride;
    sa.out_bstride = out_bstride;
    if (fused_on_ws(p, i)) return launch_ws(p->fused_op, sa, fl.q, s);
    if (n_images != 1) return hipErrorInvalidValue;
    return launch_stream(p->fused_op, sa, fl.q, s);
}

}  // namespace

namespace gabor {

std::vector<BatchFreq> batch_freq_table(const gabor_plan_s* p)
{
    std::vector<BatchFreq> freqs(p->O);
    for (int f = 0; f < p->O; ++f) {
        const FreqLaunch& fl = p->launches[f];
        BatchFreq& bf = freqs[f];
        bf.R = p->freqs[f].R;
        bf.seg_rows = fl.seg_rows;
        bf.in_scale = fl.in_scale;
        bf.mid_scale = fl.mid_scale;
        bf.out_scale = fl.out_scale;
        bf.tap_scale[0] = fl.tap_scale[0];
        bf.tap_scale[1] = fl.tap_scale[1];
        bf.q = fl.q;
    }
    return freqs;
}

}  // namespace gabor

namespace gabor {

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

int kind_index(gabor_plan p, const std::string& name, int64_t macs, int64_t bytes)
{
    for (size_t i = 0; i < p->kind_names.size(); ++i)
        if (p->kind_names[i] == name) return (int)i;
    p->kind_names.push_back(name);
    gabor_kernel_stat st{};
    std::strncpy(st.name, name.c_str(), sizeof(st.name) - 1);
    st.real_macs = macs;
    st.bytes = bytes;
    p->stats.push_back(st);
    return (int)p->kind_names.size() - 1;
}

LaunchTimer::LaunchTimer(gabor_plan plan, hipStream_t stream, const std::string& name, int64_t macs, int64_t bytes,
                         bool enabled)
    : p(plan), s(stream)
{
    if (!p->prof || !enabled) return;
    kind = kind_index(p, name, macs, bytes);
    a = take_event(p);
    b = take_event(p);
    if (a && b && hipEventRecord(a, s) == hipSuccess) return;
    if (a) p->event_pool.push_back(a);
    if (b) p->event_pool.push_back(b);
    a = b = nullptr;
}

LaunchTimer::~LaunchTimer()
{
    if (!a) return;
    if (hipEventRecord(b, s) == hipSuccess) p->pending.push_back({kind, a, b});
    else {
        p->event_pool.push_back(a);
        p->event_pool.push_back(b);
    }
}

}  // namespace gabor

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
    // LIBGABOR_ALGO=twopass selects the FP32 vector-ALU two-pass kernels
    // (comparison and testing); the default runs the fused kernel wherever
    // the band fits it.
    const char* algo_env = std::getenv("LIBGABOR_ALGO");
    const int algo = (algo_env && std::strcmp(algo_env, "twopass") == 0) ? ALGO_TWOPASS : ALGO_AUTO;

    gabor_plan p = new (std::nothrow) gabor_plan_s;
    if (!p) return GABOR_ERR_OUT_OF_MEMORY;
    p->H = height;
    p->W = width;
    p->O = n_freq;
    p->N = n_orient;
    p->boundary = boundary;
    p->precision = precision;
    // LIBGABOR_NO_GRAPH=1 submits every apply launch by launch (comparison
    // and testing); the default replays a cached graph of the apply.
    p->use_graphs = !env_flag("LIBGABOR_NO_GRAPH");
    // LIBGABOR_KERNEL=stream keeps every fused frequency on the four-wave
    // streaming kernel (comparison and testing); the default runs the
    // wave-specialised kernel wherever its quarter is built.
    {
        const char* k_env = std::getenv("LIBGABOR_KERNEL");
        p->use_ws = !(k_env && std::strcmp(k_env, "stream") == 0);
    }
    switch (precision) {
        case GABOR_PREC_FP32: p->fused_op = FUSED_F32; break;
        case GABOR_PREC_BF16_SPLIT: p->fused_op = FUSED_BF16X3; break;
        case GABOR_PREC_FP16_SPLIT: p->fused_op = FUSED_F16X3; break;
        case GABOR_PREC_BF16: p->fused_op = FUSED_BF16; break;
        case GABOR_PREC_FP16: p->fused_op = FUSED_F16; break;
    }

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

        // Pair orientations (Eq. (13)-(16)): one vertical job per horizontal
        // result, producing theta and, when present, pi - theta.
        std::vector<char> used(n_orient, 0);
        std::vector<ColJob> fjobs;
        std::vector<double> fwc, fws;
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
            p->col_macs += (int64_t)((jb.c_real ? 1 : 2) * (jb.j_real ? 1 : 2)) * fd.K * npix;
            p->row_macs += (int64_t)(jb.j_real ? 1 : 2) * fd.K * npix;
            p->n_col_passes += 1;
            p->n_row_passes += 1;
            fjobs.push_back(jb);
            fwc.push_back(wc);
            fws.push_back(ws);
        }

        // Adjoint jobs: reversed taps k(R - T) of both passes, zero-padded to Kp.
        p->adj_first.push_back((int)p->ajobs.size());
        for (size_t j = 0; j < fjobs.size(); ++j) {
            AdjJob aj{};
            aj.R = fd.R;
            aj.Kp = fd.Kp;
            aj.out_a = fjobs[j].out_a;
            aj.out_b = fjobs[j].out_b;
            aj.j_real = fjobs[j].j_real;
            aj.c_real = fjobs[j].c_real;
            aj.tap_off = (int)taps.size();
            const double w4[4] = {fwc[j], fwc[j], fws[j], fws[j]};
            for (int set = 0; set < 4; ++set)
                for (int T = 0; T < fd.Kp; ++T) {
                    double v = 0.0;
                    if (T < fd.K) {
                        const int t = fd.R - T;
                        v = S[T] * ((set & 1) ? std::sin(w4[set] * t) : std::cos(w4[set] * t));
                    }
                    taps.push_back((float)v);
                }
            p->ajobs.push_back(aj);
            p->adj_max_kp = std::max(p->adj_max_kp, fd.Kp);
            p->adj_row_macs += (int64_t)(aj.j_real ? 2 : 4) * fd.K * npix;
            p->adj_col_macs += (int64_t)(aj.c_real ? 1 : 2) * fd.K * npix;
        }

        // The fused kernel addresses the image and each output plane through
        // 32-bit buffer offsets: planes of at most 2^27 pixels (2^30 bytes).
        int64_t f_row_macs = 0, f_col_macs = 0, f_outs = 0;
        for (const ColJob& jb : fjobs) {
            f_row_macs += (int64_t)(jb.j_real ? 1 : 2) * fd.K * npix;
            f_col_macs += (int64_t)((jb.c_real ? 1 : 2) * (jb.j_real ? 1 : 2)) * fd.K * npix;
            f_outs += (jb.out_b >= 0 ? 2 : 1) * npix;
        }
        // the wave-specialised kernel's quarter where it covers R (for FP32
        // beyond R = 56 a contraction 16 rather than 32 rows longer than the
        // band), else the four-wave kernel's
        int q = stream_quarter(p->fused_op, fd.R);
        if (p->use_ws && ws_supported(p->fused_op, ws_quarter(p->fused_op, fd.R))) q = ws_quarter(p->fused_op, fd.R);
        const bool fused = q <= kStreamMaxQuarter && algo != ALGO_TWOPASS && npix <= (int64_t(1) << 27);
        // Frequencies outside the fused kernel's range run the FP32 two-pass
        // kernels whatever the requested precision (never less accurate).
        FreqLaunch fl{};
        fl.fused = fused;
        fl.q = q;
        // fused: read the image once, write every output once;
        // two-pass vertical: read the J planes, write the outputs
        fl.macs = fused ? f_row_macs + f_col_macs : f_col_macs;
        fl.bytes = fused ? 4 * npix + 8 * f_outs : 8 * (int64_t)fjobs.size() * npix + 8 * f_outs;
        fl.in_scale = fl.mid_scale = fl.out_scale = fl.tap_scale[0] = fl.tap_scale[1] = 1.0f;
        if (fused) {
            // Strip segments at least four times the lead-in, so that the
            // lead-in recomputation stays under a quarter of the J rows.
            const int L = 4 * q;
            fl.seg_rows = std::max(128, 4 * L);
            if (fl.seg_rows > height) fl.seg_rows = (height + 15) / 16 * 16;
            if (p->fused_op == FUSED_F16 || p->fused_op == FUSED_F16X3) {
                // float16 range: image scaled by 2^8 (|f| <= 128 stays below
                // 2^15), taps by the power of two that brings S(0) to
                // [2^13, 2^14); results scaled back exactly.
                const int kt = 13 - (int)std::floor(std::log2(S[fd.R]));
                const float ts = std::ldexp(1.0f, kt);
                fl.in_scale = 256.0f;
                fl.tap_scale[0] = fl.tap_scale[1] = ts;
                fl.mid_scale = 1.0f / ts;
                fl.out_scale = 1.0f / (256.0f * ts);
            }
            // Reversed taps krev[T] = k(R - T), zero-padded: entry m holds krev[m - 16].
            const int KT = L + 16;
            fl.first = (int)p->fjobs.size();
            for (size_t j = 0; j < fjobs.size(); ++j) {
                FusedJob f{};
                f.out_a = fjobs[j].out_a;
                f.out_b = fjobs[j].out_b;
                f.out_c = f.out_d = -1;
                f.j_real = fjobs[j].j_real;
                f.c_real = fjobs[j].c_real;
                f.tap_off = (int)taps.size();
                const double w4[4] = {fwc[j], fwc[j], fws[j], fws[j]};
                for (int set = 0; set < 4; ++set)
                    for (int m = 0; m < KT; ++m) {
                        const int T = m - 16;
                        double v = 0.0;
                        if (T >= 0 && T < fd.K) {
                            const int t = fd.R - T;
                            v = S[T] * ((set & 1) ? std::sin(w4[set] * t) : std::cos(w4[set] * t));
                        }
                        taps.push_back((float)v);
                    }
                p->fjobs.push_back(f);
            }
            fl.count = (int)fjobs.size();
            p->launches.push_back(fl);
            continue;
        }

        // Two-pass: vertical jobs read J planes written by horizontal groups.
        fl.first = (int)p->jobs.size();
        std::vector<RowPass> cplx, real;
        for (size_t q = 0; q < fjobs.size(); ++q) {
            ColJob jb = fjobs[q];
            // Column taps (reversed): c(R - T), d(R - T) with k(t) = S(t) e^{i ws t}.
            jb.tap_off = (int)taps.size();
            for (int T = 0; T < fd.Kp; ++T) {
                const int t = fd.R - T;
                const double s = T < fd.K ? S[T] : 0.0;   // S is symmetric: S(R-T) = S[T]
                taps.push_back((float)(s * std::cos(fws[q] * t)));
                taps.push_back((float)(s * std::sin(fws[q] * t)));
            }
            (jb.j_real ? real : cplx).push_back(RowPass{fwc[q], (bool)jb.j_real, (int)p->jobs.size()});
            p->jobs.push_back(jb);
        }
        fl.count = (int)fjobs.size();
        p->launches.push_back(fl);

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
            int64_t gm = 0;
            for (size_t m = 0; m < members.size(); ++m) {
                p->jobs[members[m]->job].plane = g.plane0 + (int)m;
                gm += (int64_t)(members[m]->real ? 1 : 2) * fd.K * npix;
            }
            p->row_group_macs.push_back(gm);
            p->n_planes += (int)members.size();
            p->row_groups.push_back(g);
            ci += g.n_cplx;
            ri += g.n_real;
        }
    }

    p->adj_first.push_back((int)p->ajobs.size());
    for (int i = 0; i < n_freq; ++i) p->order.push_back(i);
    std::stable_sort(p->order.begin(), p->order.end(),
                     [&](int a, int b) { return p->freqs[a].R > p->freqs[b].R; });

    // Device tables and workspace.
    const size_t taps_bytes = taps.size() * sizeof(float);
    const size_t jobs_bytes = p->jobs.size() * sizeof(ColJob);
    const size_t fjobs_bytes = p->fjobs.size() * sizeof(FusedJob);
    const size_t ajobs_bytes = p->ajobs.size() * sizeof(AdjJob);
    const size_t J_bytes = (size_t)p->n_planes * (size_t)npix * sizeof(float2);
    p->workspace_bytes = (int64_t)(taps_bytes + jobs_bytes + fjobs_bytes + ajobs_bytes + J_bytes);
    if (env_flag("LIBGABOR_FAIL_ALLOC")) {
        release(p);
        return GABOR_ERR_OUT_OF_MEMORY;
    }
    hipStream_t stream = (hipStream_t)hip_stream;
    hipError_t e;
    e = hipMalloc((void**)&p->d_taps, taps_bytes);
    if (e == hipSuccess && jobs_bytes) e = hipMalloc((void**)&p->d_jobs, jobs_bytes);
    if (e == hipSuccess && fjobs_bytes) e = hipMalloc((void**)&p->d_fjobs, fjobs_bytes);
    if (e == hipSuccess && J_bytes) e = hipMalloc((void**)&p->d_J, J_bytes);
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_ajobs, ajobs_bytes);
    if (e != hipSuccess) {
        release(p);
        return e == hipErrorOutOfMemory ? GABOR_ERR_OUT_OF_MEMORY : GABOR_ERR_DEVICE;
    }
    if (hipMemcpyAsync(p->d_taps, taps.data(), taps_bytes, hipMemcpyHostToDevice, stream) != hipSuccess ||
        (jobs_bytes && hipMemcpyAsync(p->d_jobs, p->jobs.data(), jobs_bytes, hipMemcpyHostToDevice, stream) != hipSuccess) ||
        (fjobs_bytes && hipMemcpyAsync(p->d_fjobs, p->fjobs.data(), fjobs_bytes, hipMemcpyHostToDevice, stream) != hipSuccess) ||
        hipMemcpyAsync(p->d_ajobs, p->ajobs.data(), ajobs_bytes, hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess) {
        release(p);
        return GABOR_ERR_DEVICE;
    }
    // Kernel attributes of the wave-specialised launches, set now rather than
    // inside a graph capture of a later apply.
    for (int i = 0; i < p->O; ++i)
        if (fused_on_ws(p, i) && prepare_ws(p->fused_op, p->launches[i].q) != hipSuccess) {
            release(p);
            return GABOR_ERR_DEVICE;
        }
    if (has_small_group(p) && prepare_ws_small(p->fused_op) != hipSuccess) {
        release(p);
        return GABOR_ERR_DEVICE;
    }
    // Independent frequencies run concurrently: up to three auxiliary
    // streams beside the caller's (four hardware queues).
    const int n_conc = std::min<int>(3, (int)p->order.size() - 1);
    for (int k = 0; k < n_conc; ++k) {
        hipStream_t st = nullptr;
        hipEvent_t e1 = nullptr, e2 = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) { release(p); return GABOR_ERR_DEVICE; }
        p->aux.push_back(st);
        if (hipEventCreateWithFlags(&e1, hipEventDisableTiming) != hipSuccess) { release(p); return GABOR_ERR_DEVICE; }
        p->fork_ev.push_back(e1);
        if (hipEventCreateWithFlags(&e2, hipEventDisableTiming) != hipSuccess) { release(p); return GABOR_ERR_DEVICE; }
        p->join_ev.push_back(e2);
    }
    *out = p;
    return GABOR_OK;
}

// ---------------------------------------------------------------------------
// Recursive-smoother plan.  Coefficients of the third-order recursive
// Gaussian (van Vliet, Young and Verbeek, ICPR 1998): poles of the sigma = 2
// design, d1, d1* = 1.40098 +- 1.00236 i and d3 = 1.85132, scaled to d^(1/q)
// with q chosen (bisection) so that the variance of the causal/anti-causal
// cascade, the sum over the poles of 2 d / (d - 1)^2, equals sigma^2.
namespace {

double iir_cascade_variance(double q)
{
    const std::complex<double> d1(1.40098, 1.00236);
    const double d3 = 1.85132;
    const std::complex<double> p1 = std::pow(d1, 1.0 / q);
    const double p3 = std::pow(d3, 1.0 / q);
    const std::complex<double> t1 = 2.0 * p1 / ((p1 - 1.0) * (p1 - 1.0));
    return 2.0 * t1.real() + 2.0 * p3 / ((p3 - 1.0) * (p3 - 1.0));
}

// a[0..3] of w[m] = a0 u[m] - a1 w[m-1] - a2 w[m-2] - a3 w[m-3]
void iir_coefficients(double sigma, double* a)
{
    double lo = 1e-3, hi = 1e4;
    for (int it = 0; it < 200; ++it) {
        const double mid = std::sqrt(lo * hi);
        if (iir_cascade_variance(mid) < sigma * sigma) lo = mid;
        else hi = mid;
    }
    const double q = std::sqrt(lo * hi);
    const std::complex<double> r1 = 1.0 / std::pow(std::complex<double>(1.40098, 1.00236), 1.0 / q);
    const double r3 = 1.0 / std::pow(1.85132, 1.0 / q);
    // (1 - r1 z^-1)(1 - conj(r1) z^-1)(1 - r3 z^-1) = 1 + a1 z^-1 + a2 z^-2 + a3 z^-3
    const double c1 = -2.0 * r1.real(), c2 = std::norm(r1);
    a[1] = c1 - r3;
    a[2] = c2 - c1 * r3;
    a[3] = -c2 * r3;
    a[0] = 1.0 + a[1] + a[2] + a[3];
}

// (cos, sin)(w l) for l = -T .. n + T - 1, the phase reduced in FP64
void push_twiddles(std::vector<float2>& tw, double w, int n, int T)
{
    const double two_pi = 2.0 * kPi;
    for (int l = -T; l < n + T; ++l) {
        double ph = std::fmod(w * (double)l, two_pi);
        double c, s;
        exact_cos_sin(ph, &c, &s);
        tw.push_back(make_float2((float)c, (float)s));
    }
}

}  // namespace

extern "C" gabor_status gabor_bank_plan_iir(gabor_plan* out, int32_t height, int32_t width, int32_t n_freq,
                                            const double* omega, const double* sigma, int32_t n_orient,
                                            const double* theta, gabor_boundary boundary, void* hip_stream)
{
    if (!out) return GABOR_ERR_INVALID_ARG;
    *out = nullptr;
    if (height <= 0 || width <= 0 || n_freq <= 0 || n_orient <= 0 || !omega || !sigma) return GABOR_ERR_INVALID_ARG;
    if (boundary != GABOR_BOUNDARY_ZERO && boundary != GABOR_BOUNDARY_MIRROR) return GABOR_ERR_INVALID_ARG;
    for (int i = 0; i < n_freq; ++i)
        if (!std::isfinite(omega[i]) || !std::isfinite(sigma[i]) || !(sigma[i] > 0.0)) return GABOR_ERR_INVALID_ARG;
    if (theta)
        for (int k = 0; k < n_orient; ++k)
            if (!std::isfinite(theta[k])) return GABOR_ERR_INVALID_ARG;
    if (height > 65535 || width > 65535) return GABOR_ERR_UNSUPPORTED;
    for (int i = 0; i < n_freq; ++i)
        if (sigma[i] < 0.5 || sigma[i] > 1000.0) return GABOR_ERR_UNSUPPORTED;
    gabor_plan p = new (std::nothrow) gabor_plan_s;
    if (!p) return GABOR_ERR_OUT_OF_MEMORY;
    p->iir = true;
    p->H = height;
    p->W = width;
    p->O = n_freq;
    p->N = n_orient;
    p->boundary = boundary;
    p->precision = GABOR_PREC_FP32;
    const int64_t npix = (int64_t)height * width;
    std::vector<double> cs(n_orient), sn(n_orient);
    for (int k = 0; k < n_orient; ++k) {
        const double th = theta ? theta[k] : kPi * (double)k / (double)n_orient;
        exact_cos_sin(th, &cs[k], &sn[k]);
    }
    std::vector<IirJob> hj, vj;
    std::vector<float2> tw;
    // Chunk length of a line of n + 2T samples and the state map across a
    // whole chunk, A^lc, in FP64 (A is the companion matrix of the
    // recursion acting on the state (w[m], w[m-1], w[m-2])).
    auto set_chunks = [](IirJob& j, const double* a, int chunks, int lc) {
        const int ext = j.n + 2 * j.T;
        j.lc = lc > 0 ? lc : (ext + chunks - 1) / chunks;
        double P[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
        const double A[9] = {-a[1], -a[2], -a[3], 1, 0, 0, 0, 1, 0};
        for (int k = 0; k < j.lc; ++k) {
            double Q[9];
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c)
                    Q[3 * r + c] = A[3 * r] * P[c] + A[3 * r + 1] * P[3 + c] + A[3 * r + 2] * P[6 + c];
            for (int q = 0; q < 9; ++q) P[q] = Q[q];
        }
        for (int q = 0; q < 9; ++q) j.apow[q] = P[q];
        for (int k = 0; k < 5; ++k) {                     // repeated squares of A^lc
            double Q[9];
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c)
                    Q[3 * r + c] = P[3 * r] * P[c] + P[3 * r + 1] * P[3 + c] + P[3 * r + 2] * P[6 + c];
            for (int q = 0; q < 9; ++q) P[q] = j.apow2[k][q] = Q[q];
        }
    };
    std::vector<int> h_of_v;                                  // horizontal job feeding each vertical job
    std::vector<std::array<double, 4>> h_coef, v_coef;        // recursion coefficients per job
    int64_t h_scr = 0, v_scr = 0;
    for (int i = 0; i < n_freq; ++i) {
        double a[4];
        iir_coefficients(sigma[i], a);
        const int T = (int)std::ceil(6.0 * sigma[i]) + 3;
        FreqDesc fd{};
        fd.R = T;
        fd.K = 2 * T + 1;
        fd.Kp = fd.K;
        p->freqs.push_back(fd);
        std::vector<char> used(n_orient, 0);
        for (int n = 0; n < n_orient; ++n) {
            if (used[n]) continue;
            used[n] = 1;
            int partner = -1;
            for (int m = n + 1; m < n_orient && !(omega[i] * cs[n] == 0.0); ++m)
                if (!used[m] && std::fabs(cs[m] + cs[n]) < kPairTol && std::fabs(sn[m] - sn[n]) < kPairTol) {
                    partner = m;
                    used[m] = 1;
                    break;
                }
            IirJob h{};
            h.in_complex = 0;
            h.n = width;
            h.cols = height;
            h.T = T;
            h.in_stride = height;
            h.out_stride = height;
            h.tw_off = (int)tw.size();
            for (int c = 0; c < 4; ++c) h.a[c] = (float)a[c];
            h_coef.push_back({a[0], a[1], a[2], a[3]});
            push_twiddles(tw, omega[i] * cs[n], width, T);
            h_scr += (int64_t)(width + 2 * T) * height;
            const int hidx = (int)hj.size();
            hj.push_back(h);
            const int vtw = (int)tw.size();
            push_twiddles(tw, omega[i] * sn[n], height, T);
            for (int side = 0; side < (partner >= 0 ? 2 : 1); ++side) {
                IirJob v{};
                v.in_complex = 1;
                v.conj = side;
                v.n = height;
                v.cols = width;
                v.T = T;
                v.in_stride = width;
                v.out_stride = width;
                v.tw_off = vtw;
                v.out_plane = i * n_orient + (side ? partner : n);
                for (int c = 0; c < 4; ++c) v.a[c] = (float)a[c];
                v_coef.push_back({a[0], a[1], a[2], a[3]});
                v_scr += (int64_t)(height + 2 * T) * width;
                vj.push_back(v);
                h_of_v.push_back(hidx);
            }
            p->n_row_passes += 1;
            p->n_col_passes += partner >= 0 ? 2 : 1;
            p->row_macs += 16 * npix;                       // two real recursions of 4 taps, each way
            p->col_macs += (int64_t)(partner >= 0 ? 2 : 1) * 16 * npix;
        }
    }
    p->n_ihj = (int)hj.size();
    p->n_ivj = (int)vj.size();
    // Chunking per pass: kIirRegChunks chunks for the register kernel when
    // every chunk fits it, else kIirChunks for the scratch-plane kernel
    // (which alone needs the scratch plane).
    // The register kernel takes one chunk length for the whole pass (the
    // longest line's, rounded up to a multiple of 8), every line padded in
    // front to kIirRegChunks chunks of it.
    auto chunk_pass = [&](std::vector<IirJob>& jobs, const std::vector<std::array<double, 4>>& coef, bool* reg,
                          int32_t* max_lc) {
        int longest = 0;
        for (const IirJob& j : jobs) longest = std::max(longest, j.n + 2 * j.T);
        const int lc = ((longest + kIirRegChunks - 1) / kIirRegChunks + 7) / 8 * 8;
        *reg = lc <= kIirRegMaxChunk;
        *max_lc = 0;
        for (size_t k = 0; k < jobs.size(); ++k) {
            if (*reg) set_chunks(jobs[k], coef[k].data(), kIirRegChunks, lc);
            else set_chunks(jobs[k], coef[k].data(), kIirChunks, 0);
            *max_lc = std::max(*max_lc, jobs[k].lc);
        }
    };
    chunk_pass(hj, h_coef, &p->iir_reg_h, &p->iir_lc_h);
    chunk_pass(vj, v_coef, &p->iir_reg_v, &p->iir_lc_v);
    if (p->iir_reg_h) h_scr = 0;
    if (p->iir_reg_v) v_scr = 0;
    p->iir_rows_h = p->iir_reg_h && p->iir_lc_h <= kIirRowChunk;
    const size_t scr = (size_t)std::max(h_scr, v_scr) * sizeof(float2);
    const size_t plane2 = (size_t)npix * sizeof(float2);
    const size_t jt_bytes = p->iir_rows_h ? 0 : hj.size() * plane2;
    p->workspace_bytes = (int64_t)(scr + jt_bytes + hj.size() * plane2 + npix * sizeof(float) +
                                   tw.size() * sizeof(float2) + (hj.size() + vj.size()) * sizeof(IirJob));
    if (env_flag("LIBGABOR_FAIL_ALLOC")) {
        release(p);
        return GABOR_ERR_OUT_OF_MEMORY;
    }
    hipError_t e = scr ? hipMalloc((void**)&p->d_iscr, scr) : hipSuccess;
    if (e == hipSuccess && jt_bytes) e = hipMalloc((void**)&p->d_iJT, jt_bytes);
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_iJ, hj.size() * plane2);
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_ifT, npix * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_itw, tw.size() * sizeof(float2));
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_ihj, hj.size() * sizeof(IirJob));
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_ivj, vj.size() * sizeof(IirJob));
    if (e != hipSuccess) {
        release(p);
        return e == hipErrorOutOfMemory ? GABOR_ERR_OUT_OF_MEMORY : GABOR_ERR_DEVICE;
    }
    // device pointers of the job tables: scratch slices, J planes (written
    // as rows, or transposed and turned back)
    int64_t off = 0;
    for (size_t j = 0; j < hj.size(); ++j) {
        hj[j].in = p->d_ifT;
        hj[j].scratch = h_scr ? p->d_iscr + off : nullptr;
        if (p->iir_rows_h) {
            hj[j].out = p->d_iJ + (int64_t)j * npix;
            hj[j].out_rows = 1;
            hj[j].out_stride = width;
        } else {
            hj[j].out = p->d_iJT + (int64_t)j * npix;
        }
        off += (int64_t)(hj[j].n + 2 * hj[j].T) * hj[j].cols;
    }
    off = 0;
    for (size_t j = 0; j < vj.size(); ++j) {
        vj[j].in = p->d_iJ + (int64_t)h_of_v[j] * npix;
        vj[j].scratch = v_scr ? p->d_iscr + off : nullptr;
        vj[j].out = nullptr;
        off += (int64_t)(vj[j].n + 2 * vj[j].T) * vj[j].cols;
    }
    hipStream_t stream = (hipStream_t)hip_stream;
    if (hipMemcpyAsync(p->d_itw, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipMemcpyAsync(p->d_ihj, hj.data(), hj.size() * sizeof(IirJob), hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipMemcpyAsync(p->d_ivj, vj.data(), vj.size() * sizeof(IirJob), hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess) {
        release(p);
        return GABOR_ERR_DEVICE;
    }
    *out = p;
    return GABOR_OK;
}

namespace {

// Every launch of one apply on `stream` (fork to the plan's streams, join
// back), arguments already checked.
gabor_status apply_eager(gabor_plan p, const float* d_image, int64_t row_stride_elems, void* d_out,
                         hipStream_t stream)
{
    if (p->iir) {
        const int64_t npix = (int64_t)p->H * p->W;
        LaunchTimer tm(p, stream, "iir_fp32", p->row_macs + p->col_macs, 4 * npix + 8 * (int64_t)p->O * p->N * npix);
        return launch_iir(d_image, row_stride_elems, p->H, p->W, p->boundary, p->d_ifT, p->d_ihj, p->n_ihj,
                          p->iir_lc_h, p->iir_reg_h, p->iir_rows_h, p->d_iJT, p->d_iJ, p->d_ivj, p->n_ivj, p->iir_lc_v, p->iir_reg_v,
                          p->d_itw, (float2*)d_out, stream) == hipSuccess
                   ? GABOR_OK
                   : GABOR_ERR_DEVICE;
    }
    for (size_t gi = 0; gi < p->row_groups.size(); ++gi) {
        const RowGroup& g = p->row_groups[gi];
        const int64_t npix = (int64_t)p->H * p->W;
        LaunchTimer tm(p, stream, "row_fp32_r" + std::to_string(p->freqs[g.freq].R), p->row_group_macs[gi],
                       4 * npix + 8 * (int64_t)(g.n_cplx + g.n_real) * npix);
        if (launch_row_fp32(d_image, row_stride_elems, p->H, p->W, p->boundary, p->freqs[g.freq], g,
                            p->d_taps, p->d_J, stream) != hipSuccess)
            return GABOR_ERR_DEVICE;
    }
    // Heaviest frequencies (largest R) first; launch j > 0 goes to
    // auxiliary stream (j - 1) mod n, which first waits for the work already
    // queued on the caller's stream (the image may have just been written).
    const int n_aux = (int)p->aux.size();
    if (n_aux > 0 && hipEventRecord(p->fork_ev[0], stream) != hipSuccess) return GABOR_ERR_DEVICE;
    for (int k = 0; k < n_aux; ++k)
        if (hipStreamWaitEvent(p->aux[k], p->fork_ev[0], 0) != hipSuccess) return GABOR_ERR_DEVICE;
    for (size_t j = 0; j < p->order.size(); ++j) {
        const int i = p->order[j];
        const FreqLaunch& fl = p->launches[i];
        hipStream_t ls = (j == 0 || n_aux == 0) ? stream : p->aux[(j - 1) % n_aux];
        if (fl.fused) {
            LaunchTimer tm(p, ls,
                           std::string(fused_on_ws(p, i) ? kWsNames[p->fused_op] : kFusedNames[p->fused_op]) +
                               "_r" + std::to_string(p->freqs[i].R),
                           fl.macs, fl.bytes);
            if (launch_fused_freq(p, i, d_image, row_stride_elems, d_out, fl.seg_rows, ls) != hipSuccess)
                return GABOR_ERR_DEVICE;
        } else {
            LaunchTimer tm(p, ls, "col_fp32_r" + std::to_string(p->freqs[i].R), fl.macs, fl.bytes);
            if (launch_col_fp32(p->d_J, p->H, p->W, p->boundary, p->freqs[i], p->d_jobs + fl.first,
                                fl.count, p->d_taps, (float2*)d_out, ls) != hipSuccess)
                return GABOR_ERR_DEVICE;
        }
    }
    for (int k = 0; k < n_aux; ++k) {
        if (hipEventRecord(p->join_ev[k], p->aux[k]) != hipSuccess ||
            hipStreamWaitEvent(stream, p->join_ev[k], 0) != hipSuccess)
            return GABOR_ERR_DEVICE;
    }
    return GABOR_OK;
}

}  // namespace

namespace gabor {

void clear_apply_graphs(gabor_plan_s* p)
{
    for (auto& g : p->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.batch) (void)gabor_batch_destroy(g.batch);
    }
    p->graphs.clear();
}

}  // namespace gabor

namespace {

// A graph of one batch apply, captured on the plan's capture stream (the
// fork, joins and launches become graph dependencies and nodes); null if
// capture fails.
hipGraphExec_t capture_batch(gabor_plan p, gabor_batch batch)
{
    if (!p->cap && hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess) {
        p->cap = nullptr;
        return nullptr;
    }
    if (hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
    const gabor_status st = gabor_batch_apply(batch, p->cap);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(p->cap, &graph);
    if (st != GABOR_OK || e != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        return nullptr;
    }
    hipGraphExec_t exec = nullptr;
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) exec = nullptr;
    (void)hipGraphDestroy(graph);
    return exec;
}

// Cached applies per plan: the few buffer triples a caller alternates between.
constexpr size_t kApplyGraphs = 4;

}  // namespace

extern "C" gabor_status gabor_bank_apply(gabor_plan p, const float* d_image, int64_t row_stride_elems,
                                         void* d_out, void* hip_stream)
{
    if (!p || !d_image || !d_out) return GABOR_ERR_INVALID_ARG;
    if (row_stride_elems < p->W) return GABOR_ERR_INVALID_ARG;
    if (!p->fjobs.empty() && (int64_t)(p->H - 1) * row_stride_elems + p->W >= (int64_t(1) << 30))
        return GABOR_ERR_UNSUPPORTED;   // image span past the 32-bit buffer offsets of the fused kernel
    hipStream_t stream = (hipStream_t)hip_stream;
    // An apply runs as a one-image batch of the plan: one launch per operand
    // quarter over a tile table sorted by decreasing cost (rather than one
    // launch per frequency), replayed from a cached graph: submitting it
    // launch by launch costs about 15 runtime calls on the host, as long as
    // a 16-bit apply's GPU work, and the graph is one.  The batch and graph
    // are built at the first apply on a (image, stride, output, schedule);
    // building synchronises the stream.  Profiled applies run the batch
    // launch by launch (events per launch); applies on a stream that is itself
    // being captured, plans with two-pass frequencies (whose batches would hold
    // J planes of their own) and recursive-smoother plans run the
    // per-frequency launches directly.
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (!p->use_graphs || p->iir || !p->row_groups.empty() || hipStreamIsCapturing(stream, &cs) != hipSuccess ||
        cs != hipStreamCaptureStatusNone)
        return apply_eager(p, d_image, row_stride_elems, d_out, stream);
    std::vector<int> segs(p->launches.size());
    for (size_t i = 0; i < segs.size(); ++i) segs[i] = p->launches[i].seg_rows;
    size_t k = 0;
    for (; k < p->graphs.size(); ++k)
        if (p->graphs[k].img == d_image && p->graphs[k].stride == row_stride_elems && p->graphs[k].out == d_out &&
            p->graphs[k].segs == segs)
            break;
    if (k < p->graphs.size()) {
        std::rotate(p->graphs.begin() + (long)k, p->graphs.begin() + (long)k + 1, p->graphs.end());  // most recent last
    } else {
        gabor_batch b = nullptr;
        const int32_t h = p->H, w = p->W;
        const float* const imgs[1] = {d_image};
        void* const outs[1] = {d_out};
        if (gabor_batch_create(&b, p, 1, imgs, &h, &w, &row_stride_elems, outs, hip_stream) != GABOR_OK)
            return apply_eager(p, d_image, row_stride_elems, d_out, stream);
        if (p->graphs.size() >= kApplyGraphs) {
            if (p->graphs.front().exec) (void)hipGraphExecDestroy(p->graphs.front().exec);
            (void)gabor_batch_destroy(p->graphs.front().batch);
            p->graphs.erase(p->graphs.begin());
        }
        p->graphs.push_back({d_image, row_stride_elems, d_out, std::move(segs), b, nullptr});
    }
    auto& g = p->graphs.back();
    if (p->prof) return gabor_batch_apply(g.batch, hip_stream);
    if (!g.exec) g.exec = capture_batch(p, g.batch);
    if (!g.exec) return gabor_batch_apply(g.batch, hip_stream);
    return hipGraphLaunch(g.exec, stream) == hipSuccess ? GABOR_OK : GABOR_ERR_DEVICE;
}

extern "C" gabor_status gabor_bank_apply_batched(gabor_plan p, const float* d_images, int32_t n_images,
                                                 int64_t image_stride_elems, int64_t row_stride_elems, void* d_out,
                                                 void* hip_stream)
{
    if (!p || n_images < 0) return GABOR_ERR_INVALID_ARG;
    if (n_images == 0) return GABOR_OK;
    if (!d_images || !d_out || row_stride_elems < p->W) return GABOR_ERR_INVALID_ARG;
    const int64_t span = (int64_t)(p->H - 1) * row_stride_elems + p->W;
    if (n_images > 1 && image_stride_elems < span) return GABOR_ERR_INVALID_ARG;
    const int64_t out_bstride = (int64_t)p->O * p->N * p->H * p->W;
    hipStream_t stream = (hipStream_t)hip_stream;
    bool one_launch = !p->iir && p->row_groups.empty();
    for (int i = 0; i < p->O; ++i) one_launch = one_launch && fused_on_ws(p, i);
    if (!one_launch) {
        // plans with two-pass or four-wave frequencies: one apply per image
        // (launch by launch: each image's buffers differ)
        if (!p->fjobs.empty() && span >= (int64_t(1) << 30)) return GABOR_ERR_UNSUPPORTED;
        for (int b = 0; b < n_images; ++b) {
            const gabor_status st = apply_eager(p, d_images + b * image_stride_elems, row_stride_elems,
                                                static_cast<float2*>(d_out) + b * out_bstride, stream);
            if (st != GABOR_OK) return st;
        }
        return GABOR_OK;
    }
    if (span >= (int64_t(1) << 30)) return GABOR_ERR_UNSUPPORTED;   // 32-bit buffer offsets per image
    // every image in each frequency's launch; the launches fork and join as in gabor_bank_apply
    const int n_aux = (int)p->aux.size();
    if (n_aux > 0 && hipEventRecord(p->fork_ev[0], stream) != hipSuccess) return GABOR_ERR_DEVICE;
    for (int k = 0; k < n_aux; ++k)
        if (hipStreamWaitEvent(p->aux[k], p->fork_ev[0], 0) != hipSuccess) return GABOR_ERR_DEVICE;
    for (size_t j = 0; j < p->order.size(); ++j) {
        const int i = p->order[j];
        const FreqLaunch& fl = p->launches[i];
        hipStream_t ls = (j == 0 || n_aux == 0) ? stream : p->aux[(j - 1) % n_aux];
        // profile name per batch size (the stat holds one launch's work)
        LaunchTimer tm(p, ls,
                       std::string(kWsNames[p->fused_op]) + "_r" + std::to_string(p->freqs[i].R) +
                           (n_images > 1 ? "_x" + std::to_string(n_images) : std::string()),
                       fl.macs * n_images, fl.bytes * n_images);
        if (launch_fused_freq(p, i, d_images, row_stride_elems, d_out, fl.seg_rows, ls, n_images, image_stride_elems,
                              out_bstride) != hipSuccess)
            return GABOR_ERR_DEVICE;
    }
    for (int k = 0; k < n_aux; ++k)
        if (hipEventRecord(p->join_ev[k], p->aux[k]) != hipSuccess ||
            hipStreamWaitEvent(stream, p->join_ev[k], 0) != hipSuccess)
            return GABOR_ERR_DEVICE;
    return GABOR_OK;
}

namespace gabor {

gabor_status adjoint_layout(const gabor_plan_s* p, AdjLayout* L)
{
    if (p->iir) return GABOR_ERR_UNSUPPORTED;
    const bool mirror = p->boundary == GABOR_BOUNDARY_MIRROR;
    if (mirror && p->O > kAdjFoldMaxFreq) return GABOR_ERR_UNSUPPORTED;
    *L = AdjLayout{};
    bool any_mfma = false;
    for (int i = 0; i < p->O; ++i) {
        const FreqLaunch& fl = p->launches[i];
        const bool m = fl.fused && fl.q <= kAdjStreamMaxQuarter;
        L->mfma.push_back(m ? 1 : 0);
        any_mfma = any_mfma || m;
        const int kp = p->freqs[i].Kp;
        if (!m && (adj_row_lds_bytes(kp) > 160 * 1024 || adj_col_lds_bytes(kp) > 160 * 1024))
            return GABOR_ERR_UNSUPPORTED;
    }
    auto align = [](int64_t b) { return (b + 255) / 256 * 256; };
    L->direct = !mirror && !any_mfma;
    if (L->direct) {
        L->bytes = align((int64_t)p->ajobs.size() * p->H * p->W * (int64_t)sizeof(float2));
        return GABOR_OK;
    }
    int64_t jc = 0;
    for (int i = 0; i < p->O; ++i) {
        const int off = mirror ? p->freqs[i].R : 0;
        const int64_t Ho = p->H + 2 * off, Wo = p->W + 2 * off;
        const int n_jobs = p->adj_first[i + 1] - p->adj_first[i];
        const int planes = L->mfma[i] ? n_jobs : 1;
        L->base.push_back(L->part_floats);
        L->planes.push_back(planes);
        L->part_floats += (int64_t)planes * Ho * Wo;
        L->jbase.push_back(L->mfma[i] ? -1 : jc);
        if (!L->mfma[i]) jc += (int64_t)n_jobs * p->H * Wo;
    }
    L->j_offset = align(L->part_floats * (int64_t)sizeof(float));
    L->bytes = align(L->j_offset + jc * (int64_t)sizeof(float2));
    return GABOR_OK;
}

gabor_status adjoint_run(gabor_plan p, const AdjLayout& L, void* ws, const void* d_grad_out, int n_images,
                         int64_t g_bstride, float* d_grad, int64_t grad_bstride, int64_t grad_row_stride_elems,
                         hipStream_t stream, bool timed)
{
    if (n_images <= 0) return GABOR_OK;
    const bool mirror = p->boundary == GABOR_BOUNDARY_MIRROR;
    const int64_t npix = (int64_t)p->H * p->W;
    const float2* G = static_cast<const float2*>(d_grad_out);
    char* wsb = static_cast<char*>(ws);
    bool all_mfma = !L.direct;
    for (char m : L.mfma) all_mfma = all_mfma && m;
    LaunchTimer tm(p, stream,
                   std::string(L.direct ? "adjoint_fp32" : all_mfma ? "adjoint_mfma_fp32" : "adjoint_mixed_fp32") +
                       (n_images > 1 ? "_x" + std::to_string(n_images) : std::string()),
                   (p->adj_row_macs + p->adj_col_macs) * n_images,
                   (8 * (int64_t)p->O * p->N * npix + 4 * npix) * n_images, timed);
    if (L.direct) {
        for (int b = 0; b < n_images; ++b)
            if (launch_adjoint(G + b * g_bstride, p->H, p->W, 0, p->d_ajobs, (int)p->ajobs.size(), p->adj_max_kp,
                               p->d_taps, reinterpret_cast<float2*>(wsb + b * L.bytes), d_grad + b * grad_bstride,
                               grad_row_stride_elems, stream) != hipSuccess)
                return GABOR_ERR_DEVICE;
        return GABOR_OK;
    }
    const int64_t part_bstride = L.bytes / (int64_t)sizeof(float);
    // the frequencies run concurrently as in the forward apply
    const int n_aux = (int)p->aux.size();
    if (n_aux > 0 && hipEventRecord(p->fork_ev[0], stream) != hipSuccess) return GABOR_ERR_DEVICE;
    for (int k = 0; k < n_aux; ++k)
        if (hipStreamWaitEvent(p->aux[k], p->fork_ev[0], 0) != hipSuccess) return GABOR_ERR_DEVICE;
    for (size_t j = 0; j < p->order.size(); ++j) {
        const int i = p->order[j];
        const FreqLaunch& fl = p->launches[i];
        hipStream_t ls = (j == 0 || n_aux == 0) ? stream : p->aux[(j - 1) % n_aux];
        const int off = mirror ? p->freqs[i].R : 0;
        const int Ho = p->H + 2 * off, Wo = p->W + 2 * off;
        if (L.mfma[i]) {
            AdjStreamArgs a{};
            a.G = G;
            a.part = reinterpret_cast<float*>(wsb) + L.base[i];
            a.H = p->H;
            a.W = p->W;
            a.R = p->freqs[i].R;
            a.off = off;
            a.Ho = Ho;
            a.Wo = Wo;
            // segments of a multiple of 32 rows unless one covers the grid
            int seg = fl.seg_rows;
            if (seg % 32 != 0 && seg < a.Ho) seg = (seg + 31) / 32 * 32;
            a.seg_rows = seg;
            a.n_xs = (a.Wo + stream_strip_width() - 1) / stream_strip_width();
            a.n_ys = (a.Ho + seg - 1) / seg;
            a.n_jobs = fl.count;
            a.jobs = p->d_fjobs + fl.first;
            a.taps = p->d_taps;
            a.n_images = n_images;
            a.g_bstride = g_bstride;
            a.part_bstride = part_bstride;
            if (launch_adjoint_stream(a, fl.q, ls) != hipSuccess) return GABOR_ERR_DEVICE;
        } else {
            const int first = p->adj_first[i], n_jobs = p->adj_first[i + 1] - first;
            for (int b = 0; b < n_images; ++b) {
                char* w = wsb + b * L.bytes;
                if (launch_adjoint(G + b * g_bstride, p->H, p->W, off, p->d_ajobs + first, n_jobs,
                                   p->freqs[i].Kp, p->d_taps, reinterpret_cast<float2*>(w + L.j_offset) + L.jbase[i],
                                   reinterpret_cast<float*>(w) + L.base[i], Wo, ls) != hipSuccess)
                    return GABOR_ERR_DEVICE;
            }
        }
    }
    for (int k = 0; k < n_aux; ++k)
        if (hipEventRecord(p->join_ev[k], p->aux[k]) != hipSuccess ||
            hipStreamWaitEvent(stream, p->join_ev[k], 0) != hipSuccess)
            return GABOR_ERR_DEVICE;
    if (mirror) {
        AdjFoldArgs fa{};
        fa.part = reinterpret_cast<const float*>(wsb);
        fa.grad = d_grad;
        fa.grad_stride = grad_row_stride_elems;
        fa.H = p->H;
        fa.W = p->W;
        fa.n_freq = p->O;
        fa.n_images = n_images;
        fa.part_bstride = part_bstride;
        fa.grad_bstride = grad_bstride;
        for (int i = 0; i < p->O; ++i) fa.f[i] = AdjFoldFreq{L.base[i], p->freqs[i].R, L.planes[i]};
        return launch_adjoint_fold_sum(fa, stream) == hipSuccess ? GABOR_OK : GABOR_ERR_DEVICE;
    }
    int total = 0;
    for (int n : L.planes) total += n;
    return launch_adjoint_sum(reinterpret_cast<const float*>(wsb), total, p->H, p->W, d_grad, grad_row_stride_elems,
                              n_images, part_bstride, grad_bstride, stream) == hipSuccess
               ? GABOR_OK
               : GABOR_ERR_DEVICE;
}

}  // namespace gabor

namespace {

// The plan's adjoint workspace, grown to at least `bytes` (after the work
// already queued on `stream`, which every adjoint call joins back to, has
// finished with the old one).
gabor_status adjoint_reserve(gabor_plan p, int64_t bytes, hipStream_t stream)
{
    if (p->d_adjW && p->adj_cap >= bytes) return GABOR_OK;
    if (env_flag("LIBGABOR_FAIL_ALLOC")) return GABOR_ERR_OUT_OF_MEMORY;
    if (p->d_adjW) {
        if (hipStreamSynchronize(stream) != hipSuccess) return GABOR_ERR_DEVICE;
        (void)hipFree(p->d_adjW);
        p->d_adjW = nullptr;
        p->workspace_bytes -= p->adj_cap;
        p->adj_cap = 0;
    }
    void* d = nullptr;
    const hipError_t e = hipMalloc(&d, (size_t)bytes);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? GABOR_ERR_OUT_OF_MEMORY : GABOR_ERR_DEVICE;
    p->d_adjW = d;
    p->adj_cap = bytes;
    p->workspace_bytes += bytes;
    return GABOR_OK;
}

// Workspace bound of one batched adjoint launch group: images beyond it run
// in further groups.
constexpr int64_t kAdjBatchBytes = int64_t(1) << 30;

}  // namespace

extern "C" gabor_status gabor_bank_apply_adjoint(gabor_plan p, const void* d_grad_out, float* d_grad_image,
                                                 int64_t grad_row_stride_elems, void* hip_stream)
{
    if (!p || !d_grad_out || !d_grad_image) return GABOR_ERR_INVALID_ARG;
    if (grad_row_stride_elems < p->W) return GABOR_ERR_INVALID_ARG;
    AdjLayout L;
    gabor_status st = adjoint_layout(p, &L);
    if (st != GABOR_OK) return st;
    hipStream_t stream = (hipStream_t)hip_stream;
    // the plan keeps its adjoint workspace from the first call on
    if ((st = adjoint_reserve(p, L.bytes, stream)) != GABOR_OK) return st;
    return adjoint_run(p, L, p->d_adjW, d_grad_out, 1, 0, d_grad_image, 0, grad_row_stride_elems, stream, true);
}

extern "C" gabor_status gabor_bank_apply_adjoint_batched(gabor_plan p, const void* d_grad_out, int32_t n_images,
                                                         float* d_grad_images, int64_t grad_image_stride_elems,
                                                         int64_t grad_row_stride_elems, void* hip_stream)
{
    if (!p || n_images < 0) return GABOR_ERR_INVALID_ARG;
    if (n_images == 0) return GABOR_OK;
    if (!d_grad_out || !d_grad_images) return GABOR_ERR_INVALID_ARG;
    if (grad_row_stride_elems < p->W ||
        (n_images > 1 && grad_image_stride_elems < (int64_t)(p->H - 1) * grad_row_stride_elems + p->W))
        return GABOR_ERR_INVALID_ARG;
    AdjLayout L;
    gabor_status st = adjoint_layout(p, &L);
    if (st != GABOR_OK) return st;
    hipStream_t stream = (hipStream_t)hip_stream;
    // LIBGABOR_ADJ_BATCH_BYTES lowers the group bound (tests of the grouping)
    int64_t cap = kAdjBatchBytes;
    if (const char* v = std::getenv("LIBGABOR_ADJ_BATCH_BYTES")) cap = std::max<int64_t>(1, std::atoll(v));
    const int chunk = (int)std::max<int64_t>(1, std::min<int64_t>(n_images, cap / L.bytes));
    if ((st = adjoint_reserve(p, (int64_t)chunk * L.bytes, stream)) != GABOR_OK) return st;
    const int64_t g_bstride = (int64_t)p->O * p->N * p->H * p->W;
    const float2* G = static_cast<const float2*>(d_grad_out);
    for (int b0 = 0; b0 < n_images; b0 += chunk) {
        const int n = std::min(chunk, n_images - b0);
        st = adjoint_run(p, L, p->d_adjW, G + b0 * g_bstride, n, g_bstride, d_grad_images + b0 * grad_image_stride_elems,
                         grad_image_stride_elems, grad_row_stride_elems, stream, true);
        if (st != GABOR_OK) return st;
    }
    return GABOR_OK;
}

// Segment heights the tuner tries for one fused launch, up to the image
// height: multiples of 32 for the four-wave kernel, of 16 for the
// wave-specialised one (which also tries finer steps).
static std::vector<int> seg_candidates(int H, int q, bool ws)
{
    const int hmax = (H + 15) / 16 * 16;
    std::vector<int> c;
    std::vector<int> v = {64, 128, 192, 256, 384, 512, 16 * q, 32 * q};
    if (ws) v.insert(v.end(), {96, 160, 224, 320, 448, 640, 768, hmax});
    for (int x : v) {
        const int s = std::min(x, hmax);
        if (s >= 16 && (ws || s % 32 == 0 || s == hmax) && std::find(c.begin(), c.end(), s) == c.end())
            c.push_back(s);
    }
    std::sort(c.begin(), c.end());
    return c;
}

// Median of reps timed applies (after one untimed one), in ms; sets *rc on
// a device error.
// Whole-apply time of the current schedule: one apply that builds its batch
// and graph, then the median over `reps` bursts of kTuneBurst back-to-back
// applies (the rate of repeated applies, with the launch latency of one
// overlapping the work of the one before, as a caller applying the bank in a
// loop sees it).
constexpr int kTuneBurst = 8;
static double time_apply(gabor_plan p, const float* d_image, int64_t row_stride_elems, void* d_out, void* hip_stream,
                         int reps, hipEvent_t a, hipEvent_t b, gabor_status* rc)
{
    hipStream_t stream = (hipStream_t)hip_stream;
    if (gabor_bank_apply(p, d_image, row_stride_elems, d_out, hip_stream) != GABOR_OK ||
        hipStreamSynchronize(stream) != hipSuccess) {
        *rc = GABOR_ERR_DEVICE;
        return 1e30;
    }
    std::vector<float> t;
    for (int r = 0; r < reps; ++r) {
        float ms = 0.0f;
        bool ok = hipEventRecord(a, stream) == hipSuccess;
        for (int k = 0; ok && k < kTuneBurst; ++k)
            ok = gabor_bank_apply(p, d_image, row_stride_elems, d_out, hip_stream) == GABOR_OK;
        if (!ok || hipEventRecord(b, stream) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
            hipEventElapsedTime(&ms, a, b) != hipSuccess) {
            *rc = GABOR_ERR_DEVICE;
            return 1e30;
        }
        t.push_back(ms / kTuneBurst);
    }
    std::nth_element(t.begin(), t.begin() + t.size() / 2, t.end());
    return t[t.size() / 2];
}

extern "C" gabor_status gabor_bank_autotune(gabor_plan p, const float* d_image, int64_t row_stride_elems,
                                            void* d_out, int32_t reps, void* hip_stream)
{
    if (!p || !d_image || !d_out || reps < 1) return GABOR_ERR_INVALID_ARG;
    if (row_stride_elems < p->W) return GABOR_ERR_INVALID_ARG;
    if (p->iir) return GABOR_OK;                                 // nothing to tune
    if (!p->fjobs.empty() && (int64_t)(p->H - 1) * row_stride_elems + p->W >= (int64_t(1) << 30))
        return GABOR_ERR_UNSUPPORTED;
    hipStream_t stream = (hipStream_t)hip_stream;
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess) return GABOR_ERR_DEVICE;
    if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return GABOR_ERR_DEVICE; }
    gabor_status rc = GABOR_OK;
    for (int i = 0; i < p->O && rc == GABOR_OK; ++i) {
        FreqLaunch& fl = p->launches[i];
        if (!fl.fused) continue;
        double best = 1e30;
        int best_seg = fl.seg_rows;
        for (int seg : seg_candidates(p->H, fl.q, fused_on_ws(p, i))) {
            // one untimed launch, then the median of reps timed launches
            if (launch_fused_freq(p, i, d_image, row_stride_elems, d_out, seg, stream) != hipSuccess) { rc = GABOR_ERR_DEVICE; break; }
            std::vector<float> t;
            for (int r = 0; r < reps; ++r) {
                float ms = 0.0f;
                if (hipEventRecord(a, stream) != hipSuccess ||
                    launch_fused_freq(p, i, d_image, row_stride_elems, d_out, seg, stream) != hipSuccess ||
                    hipEventRecord(b, stream) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                    hipEventElapsedTime(&ms, a, b) != hipSuccess) {
                    rc = GABOR_ERR_DEVICE;
                    break;
                }
                t.push_back(ms);
            }
            if (rc != GABOR_OK) break;
            std::nth_element(t.begin(), t.begin() + t.size() / 2, t.end());
            if (t[t.size() / 2] < best) {
                best = t[t.size() / 2];
                best_seg = seg;
            }
        }
        fl.seg_rows = best_seg;
    }
    // The frequencies run concurrently in an apply, where fewer, longer
    // segments (less lead-in recomputation) can beat the per-launch optimum:
    // time the whole apply with every segment scaled by 1, 2 and 4.
    std::vector<int> per_launch(p->O);
    for (int i = 0; i < p->O; ++i) per_launch[i] = p->launches[i].seg_rows;
    auto tune_whole = [&]() -> double {
        double best_t = 1e30;
        if (rc != GABOR_OK || p->fjobs.empty()) return best_t;
        std::vector<int> base_seg(per_launch), best(per_launch);
        for (int i = 0; i < p->O; ++i) p->launches[i].seg_rows = per_launch[i];
        const int hmax = (p->H + 15) / 16 * 16;
        for (int mult : {1, 2, 4}) {
            for (int i = 0; i < p->O; ++i)
                if (p->launches[i].fused) p->launches[i].seg_rows = std::min(base_seg[i] * mult, hmax);
            const double t_med = time_apply(p, d_image, row_stride_elems, d_out, hip_stream, reps, a, b, &rc);
            if (rc != GABOR_OK) break;
            // a scaled schedule must beat the per-launch optimum clearly
            const double tm = t_med * (mult == 1 ? 1.0 : 1.01);
            if (tm < best_t) {
                best_t = tm;
                for (int i = 0; i < p->O; ++i) best[i] = p->launches[i].seg_rows;
            }
        }
        for (int i = 0; i < p->O; ++i) p->launches[i].seg_rows = best[i];
        // Coordinate descent on the whole apply: the frequencies share the
        // device, so each one's height is retimed with the others fixed
        // (two passes, heaviest frequency first).
        if (rc == GABOR_OK) best_t = time_apply(p, d_image, row_stride_elems, d_out, hip_stream, reps, a, b, &rc);
        for (int pass = 0; pass < 2 && rc == GABOR_OK; ++pass)
            for (int i : p->order) {
                if (!p->launches[i].fused || rc != GABOR_OK) continue;
                int keep = p->launches[i].seg_rows;
                for (int seg : seg_candidates(p->H, p->launches[i].q, fused_on_ws(p, i))) {
                    if (seg == keep) continue;
                    p->launches[i].seg_rows = seg;
                    const double tm = time_apply(p, d_image, row_stride_elems, d_out, hip_stream, reps, a, b, &rc);
                    if (rc != GABOR_OK) break;
                    if (tm < 0.99 * best_t) {            // a clear gain only
                        best_t = tm;
                        keep = seg;
                    }
                }
                p->launches[i].seg_rows = keep;
            }
        return best_t;
    };
    const double t_own = tune_whole();
    // The small quarters grouped into one launch (the other setting of the
    // plan's option), tuned the same way; kept only on a clear gain.
    if (rc == GABOR_OK && has_small_group(p)) {
        std::vector<int> own(p->O);
        for (int i = 0; i < p->O; ++i) own[i] = p->launches[i].seg_rows;
        const bool was = p->group_small;
        p->group_small = !was;
        clear_apply_graphs(p);
        const double t_other = tune_whole();
        if (rc == GABOR_OK && !(t_other < 0.99 * t_own)) {
            p->group_small = was;
            for (int i = 0; i < p->O; ++i) p->launches[i].seg_rows = own[i];
            clear_apply_graphs(p);
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return rc;
}

extern "C" gabor_status gabor_bank_get_tuning(gabor_plan p, int32_t* seg_rows, int32_t capacity, int32_t* n)
{
    if (!p || !n || capacity < 0 || (capacity > 0 && !seg_rows)) return GABOR_ERR_INVALID_ARG;
    *n = p->O;
    for (int i = 0; i < p->O && i < capacity; ++i) seg_rows[i] = p->launches[i].fused ? p->launches[i].seg_rows : 0;
    return GABOR_OK;
}

extern "C" gabor_status gabor_bank_set_tuning(gabor_plan p, const int32_t* seg_rows, int32_t n)
{
    if (!p || !seg_rows || n != p->O) return GABOR_ERR_INVALID_ARG;
    for (int i = 0; i < n; ++i)
        if (p->launches[i].fused && seg_rows[i] < p->H && (seg_rows[i] < 32 || seg_rows[i] % 32 != 0))
            return GABOR_ERR_INVALID_ARG;    // a segment that does not cover the image: multiple of 32 rows
    // a segment that covers the image becomes the image height rounded up
    // to 16 rows (the kernel steps 16 rows at a time)
    const int hmax = (p->H + 15) / 16 * 16;
    for (int i = 0; i < n; ++i)
        if (p->launches[i].fused) p->launches[i].seg_rows = seg_rows[i] >= p->H ? hmax : seg_rows[i];
    return GABOR_OK;
}

extern "C" gabor_status gabor_bank_get_grouping(gabor_plan p, int32_t* group_small)
{
    if (!p || !group_small) return GABOR_ERR_INVALID_ARG;
    *group_small = p->group_small ? 1 : 0;
    return GABOR_OK;
}

extern "C" gabor_status gabor_bank_set_grouping(gabor_plan p, int32_t group_small)
{
    if (!p || (group_small != 0 && group_small != 1)) return GABOR_ERR_INVALID_ARG;
    if (p->group_small != (group_small == 1)) {
        p->group_small = group_small == 1;
        clear_apply_graphs(p);                     // cached applies hold the other launches
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
