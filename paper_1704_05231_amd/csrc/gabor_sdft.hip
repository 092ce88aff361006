// Box-window 2-D sliding DFT by the circular-shift recursion, re-anchored in
// FP64.  Eq. (17) with a constant window of unit sum (the conventional SDFT
// that the paper relates Eq. (17) to, scaled by 1/(Mx My); Sec. I describes
// its recursion, which holds only for a box window):
//
//   F_{u,v}(x,y) = 1/(Mx My) sum_{j<Mx} sum_{i<My} f(x - Mx/2 + j, y - My/2 + i)
//                  exp(-i 2 pi (u j / Mx + v i / My)).
//
// With the column DFT C_v(m, y) = 1/My sum_{i<My} f(m, y - My/2 + i)
// exp(-i 2 pi v i / My) and s = x - Mx/2 the window start, shifting the
// window one column adds the entering column and drops the leaving one:
//
//   F_{u,v}(x + 1, y) = exp(i 2 pi u / Mx) (F_{u,v}(x, y) + (C_v(s + Mx) - C_v(s)) / Mx).
//
// One workgroup per (row y, bin v <= My/2) forms C_v along the row in FP64
// (direct My-term sums) in LDS.  Its waves then take the bins u in turn; each
// lane runs the recursion over a run of kRun columns, starting from a direct
// FP64 sum over the window (the anchor), so rounding never accumulates over
// more than kRun updates.  The state stays in FP64; outputs are rounded once
// to complex64 and staged through LDS so that stores are contiguous.  Every
// computed bin also gives its conjugate partner F_{Mx-u, My-v} (real input),
// so bins with v > My/2, and with u > Mx/2 on the rows v = 0 and v = My/2,
// are never computed.  Every output plane is written once.
#include <cmath>
#include <cstdint>
#include <cstring>

#include "../../include/libgabor.h"
#include "gabor_internal.h"

namespace gabor {
namespace {

constexpr int kSdftThreads = 256;
constexpr int kRun = 8;                  // columns per lane between anchors
constexpr int kSdftMaxM = 64;
constexpr int kSdftMaxW = 8192;          // row length held in LDS (FP64 column DFT)

struct SdftArgs {
    const float* img;
    int64_t stride;
    int32_t H, W, my, mx, boundary;
    int32_t wide;                        // 16-byte stores: even W and a 16-byte aligned output
    float2* out;
    double twx[2][kSdftMaxM];            // cos, sin of 2 pi k / Mx
    double twy[2][kSdftMaxM];            // cos, sin of 2 pi k / My
};

__device__ __forceinline__ int sdft_fold(int i, int n, int boundary)
{
    if ((unsigned)i < (unsigned)n) return i;
    if (boundary == 0) return -1;
    if (n == 1) return 0;
    const int p = 2 * (n - 1);
    int r = i % p;
    if (r < 0) r += p;
    return r < n ? r : p - r;
}

// LDS slot of column-DFT entry k: the low three bits are XORed with bits
// 4..6, so that any 16 consecutive lanes of a read at k = 8 lane + j (any j)
// hit 16 distinct 16-byte slots of the 256-byte bank row (the lanes' entries
// fall into nine 16-entry blocks, the two outer ones with equal XOR keys but
// in opposite halves).  A permutation within each 16-entry block; the array
// is allocated in whole blocks.
__device__ __forceinline__ int c_slot(int k) { return k ^ ((k >> 4) & 7); }

// staging slot of column t of run r (a run is one lane's kRun columns):
// rotated by r / 4 so that 32 lanes writing the same t hit distinct slots,
// and a permutation within each run, so reads of consecutive columns do too.
__device__ __forceinline__ int stage_slot(int r, int t) { return r * kRun + ((t + (r >> 2)) & (kRun - 1)); }

__global__ __launch_bounds__(kSdftThreads) void k_sdft_box(SdftArgs a)
{
    extern __shared__ double2 sdft_lds[];
    const int y = blockIdx.x, v = blockIdx.y;
    const int W = a.W, mx = a.mx, my = a.my, hx = mx / 2, hy = my / 2;
    const int tid = threadIdx.x, lane = tid & 63;
    // wave index, held in a scalar register: bins u, and with them the twiddle
    // indices, are then wave-uniform and the tables are read by scalar loads
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int n_c = (W + mx + 15) & ~15;
    double2* C = sdft_lds;                                            // C[c_slot(k)] = C_v(k - hx)
    float2* stage_all = reinterpret_cast<float2*>(C + n_c);             // one kRun x 64 block per wave
    float2* stage = stage_all + w * 64 * kRun;
    // window row i: its image row offset (or -1 outside a zero boundary) and
    // the twiddle exp(-i 2 pi v i / My) / My
    int64_t* row_off = reinterpret_cast<int64_t*>(stage_all + 4 * 64 * kRun);
    double2* row_tw = reinterpret_cast<double2*>(row_off + kSdftMaxM);
    if (tid < my) {
        const int yy = sdft_fold(y - hy + tid, a.H, a.boundary);
        row_off[tid] = yy < 0 ? -1 : (int64_t)yy * a.stride;
        const int t = (v * tid) % my;
        row_tw[tid] = make_double2(a.twy[0][t] / my, -a.twy[1][t] / my);
    }
    __syncthreads();

    // column DFT of every window column of this row, FP64
    for (int k = tid; k < W + mx; k += kSdftThreads) {
        const int xx = sdft_fold(k - hx, W, a.boundary);
        double cr = 0.0, ci = 0.0;
        if (xx >= 0) {
#pragma unroll 8
            for (int i = 0; i < my; ++i) {
                // unconditional load (row 0 stands in for rows outside a zero
                // boundary) and a select, so the unrolled loads issue together
                const int64_t ro = row_off[i];
                const float raw = a.img[(ro < 0 ? 0 : ro) + xx];
                const double f = ro < 0 ? 0.0 : (double)raw;
                const double2 tw = row_tw[i];
                cr += f * tw.x;
                ci += f * tw.y;
            }
        }
        C[c_slot(k)] = make_double2(cr, ci);
    }
    __syncthreads();

    const int64_t plane = (int64_t)a.H * W;
    const int n_runs = (W + kRun - 1) / kRun;
    const double inv_mx = 1.0 / mx;
    // Rows v = 0 and v = My/2 are their own conjugate partners: there the
    // bins u > Mx/2 are the conjugates of u < Mx/2, so only u <= Mx/2 run.
    const int vp = (my - v) % my;
    const int n_u = vp == v ? mx / 2 + 1 : mx;
    // every wave runs the same number of rounds, so the barriers line up
    const int rounds = (n_u + 3) / 4;
    for (int rd = 0; rd < rounds; ++rd) {
        const int u = 4 * rd + w;
        const bool active = u < n_u;
        const int uu = active ? u : 0;
        const double er = a.twx[0][uu], ei = a.twx[1][uu];          // exp(+i 2 pi u / Mx)
        const int pa = v * mx + uu, pb = vp * mx + (mx - uu) % mx;
        const bool partner = pb != pa;                              // else the bin is real
        float2* fa = a.out + (int64_t)pa * plane + (int64_t)y * W;
        float2* fb = a.out + (int64_t)pb * plane + (int64_t)y * W;
        for (int r0 = 0; r0 < n_runs; r0 += 64) {
            const int x0 = (r0 + lane) * kRun;
            if (active && x0 < W) {
                // anchor: F(x0) = 1/Mx sum_j C(x0 - hx + j) exp(-i 2 pi u j / Mx)
                double fr = 0.0, fi = 0.0;
                int tw = 0;
#pragma unroll 4
                for (int j = 0; j < mx; ++j) {
                    const double2 c = C[c_slot(x0 + j)];
                    const double tr = a.twx[0][tw], ti = -a.twx[1][tw];
                    fr += c.x * tr - c.y * ti;
                    fi += c.x * ti + c.y * tr;
                    tw += uu;                                         // tw = u j mod Mx
                    if (tw >= mx) tw -= mx;
                }
                fr *= inv_mx;
                fi *= inv_mx;
#pragma unroll
                for (int t = 0; t < kRun; ++t) {
                    stage[stage_slot(lane, t)] = make_float2((float)fr, (float)fi);
                    const int x = x0 + t;
                    // the state after the run's last column is the next lane's anchor
                    if (t + 1 < kRun && x + 1 < W) {
                        const double2 cin = C[c_slot(x + mx)], cout = C[c_slot(x)];
                        const double gr = fr + (cin.x - cout.x) * inv_mx, gi = fi + (cin.y - cout.y) * inv_mx;
                        fr = gr * er - gi * ei;
                        fi = gr * ei + gi * er;
                    }
                }
            }
            __syncthreads();
            // contiguous stores of the staged columns: two columns (16 bytes)
            // per lane when every column pair is 16-byte aligned
            if (active && a.wide) {
                for (int e = 2 * lane; e < 64 * kRun; e += 128) {
                    const int x = r0 * kRun + e;
                    if (x < W) {
                        const float2 v0 = stage[stage_slot(e / kRun, e % kRun)];
                        const float2 v1 = stage[stage_slot(e / kRun, e % kRun + 1)];
                        *reinterpret_cast<float4*>(fa + x) = make_float4(v0.x, v0.y, v1.x, v1.y);
                        if (partner) *reinterpret_cast<float4*>(fb + x) = make_float4(v0.x, -v0.y, v1.x, -v1.y);
                    }
                }
            } else if (active) {
                for (int e = lane; e < 64 * kRun; e += 64) {
                    const int x = r0 * kRun + e;
                    if (x < W) {
                        const float2 val = stage[stage_slot(e / kRun, e % kRun)];
                        fa[x] = val;
                        if (partner) fb[x] = make_float2(val.x, -val.y);
                    }
                }
            }
            __syncthreads();
        }
    }
}

// cos and sin of 2 pi k / M, exact at quarter turns
void sdft_table(int M, double* c, double* s)
{
    constexpr double kPi = 3.14159265358979323846264338327950288;
    for (int k = 0; k < M; ++k) {
        if ((4 * k) % M == 0) {
            static const double qc[4] = {1.0, 0.0, -1.0, 0.0}, qs[4] = {0.0, 1.0, 0.0, -1.0};
            c[k] = qc[(4 * k / M) % 4];
            s[k] = qs[(4 * k / M) % 4];
        } else {
            const double ang = 2.0 * kPi * (double)k / (double)M;
            c[k] = std::cos(ang);
            s[k] = std::sin(ang);
        }
    }
}

}  // namespace
}  // namespace gabor

using namespace gabor;

extern "C" gabor_status sdft_box_apply(const float* d_image, int32_t height, int32_t width,
                                       int64_t row_stride_elems, int32_t m_y, int32_t m_x,
                                       gabor_boundary boundary, void* d_out, void* hip_stream)
{
    if (!d_image || !d_out) return GABOR_ERR_INVALID_ARG;
    if (height <= 0 || width <= 0 || m_y <= 0 || m_x <= 0) return GABOR_ERR_INVALID_ARG;
    if (row_stride_elems < width) return GABOR_ERR_INVALID_ARG;
    if (boundary != GABOR_BOUNDARY_ZERO && boundary != GABOR_BOUNDARY_MIRROR) return GABOR_ERR_INVALID_ARG;
    if (m_y > kSdftMaxM || m_x > kSdftMaxM || width > kSdftMaxW || height > 65535) return GABOR_ERR_UNSUPPORTED;
    if ((int64_t)height * width * m_y * m_x > (int64_t(1) << 40)) return GABOR_ERR_UNSUPPORTED;
    SdftArgs a;
    std::memset(&a, 0, sizeof(a));
    a.img = d_image;
    a.stride = row_stride_elems;
    a.H = height;
    a.W = width;
    a.my = m_y;
    a.mx = m_x;
    a.boundary = boundary;
    a.out = (float2*)d_out;
    a.wide = (width % 2 == 0 && ((uintptr_t)d_out & 15) == 0) ? 1 : 0;
    sdft_table(m_x, a.twx[0], a.twx[1]);
    sdft_table(m_y, a.twy[0], a.twy[1]);
    const size_t lds = (size_t)((width + m_x + 15) & ~15) * sizeof(double2) + (size_t)4 * 64 * kRun * sizeof(float2) +
                       (size_t)kSdftMaxM * (sizeof(int64_t) + sizeof(double2));
    hipStream_t stream = (hipStream_t)hip_stream;
    static LdsLimit lim;
    if (lim.ensure((const void*)k_sdft_box, lds) != hipSuccess) return GABOR_ERR_DEVICE;
    hipLaunchKernelGGL(k_sdft_box, dim3(height, m_y / 2 + 1), dim3(kSdftThreads), lds, stream, a);
    return hipGetLastError() == hipSuccess ? GABOR_OK : GABOR_ERR_DEVICE;
}
