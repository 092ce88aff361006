// Batched bank: many images of uneven sizes through one plan (Algorithm 1 per
// image).  gabor_batch_create binds the images and outputs once and uploads
// a tile table; gabor_batch_apply then only launches, so it allocates and
// copies nothing and may be captured in a HIP graph and replayed.
//
// Frequencies on the fused kernels are grouped by operand quarter Q; each
// group is one launch over the tiles (image, job, strip segment) of every
// image, in decreasing cost.  Tile b is workgroup b (the wave-specialised
// kernel, and beyond its quarters the four-wave one), so the dispatcher
// hands out the longest tiles first and the rest as workgroups free up.
// One kernel
// over all quarters would carry the largest quarter's registers and LDS
// into every tile (measured: 185 to 256 registers with spills against 124
// to 177 per quarter), so each quarter keeps a launch of its own, except
// that the plan's grouping option puts the small quarters (whose resources
// are close) into one.  Frequencies outside the fused kernel's range run the
// FP32 two-pass kernels on the caller's stream, one launch per pass over all
// images, each image with J planes of its own in a batch-owned workspace.
#include <algorithm>
#include <array>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "gabor_plan_impl.h"

namespace {

struct BatchGroup {
    int q;                     // quarter, or 0: the small quarters in one launch
    int first_tile, n_tiles;
    int64_t weight;            // total tile steps, for ordering the launches
    std::string name;          // profile name: kernel and the radii it covers
    int64_t macs, bytes;       // algorithmic work of one launch
};

// Dispatch order of a launch's tiles: decreasing cost (the dispatcher hands
// out the longest tiles first and the rest as workgroups free up), and
// within each run of equal cost, the tiles of eight strip segments (same
// image, frequency, strip and rows: the same image rows) interleaved: the
// first tile of each of the eight, then the second of each, ...  Workgroup b
// of a launch goes to XCD b mod 8, each XCD with its own L2, so a strip
// segment's equal-cost jobs (the pairs of a frequency) then run on one XCD
// one after another instead of on three.
constexpr int kXcds = 8;
void xcd_order(std::vector<std::pair<int64_t, BatchTile>>& tl)
{
    std::stable_sort(tl.begin(), tl.end(), [](const auto& a, const auto& c) { return a.first > c.first; });
    std::vector<std::pair<int64_t, BatchTile>> out;
    out.reserve(tl.size());
    for (size_t r0 = 0; r0 < tl.size();) {
        size_t r1 = r0;
        while (r1 < tl.size() && tl[r1].first == tl[r0].first) ++r1;
        // strip segments of the run, in order of first appearance
        std::vector<std::vector<size_t>> segs;
        std::map<std::array<int32_t, 3>, size_t> index;
        for (size_t k = r0; k < r1; ++k) {
            const BatchTile& t = tl[k].second;
            const auto it = index.emplace(std::array<int32_t, 3>{t.image, t.freq, t.rest}, segs.size()).first;
            if (it->second == segs.size()) segs.emplace_back();
            segs[it->second].push_back(k);
        }
        for (size_t s0 = 0; s0 < segs.size(); s0 += kXcds) {
            const size_t s1 = std::min(segs.size(), s0 + kXcds);
            size_t most = 0;
            for (size_t k = s0; k < s1; ++k) most = std::max(most, segs[k].size());
            for (size_t j = 0; j < most; ++j)
                for (size_t k = s0; k < s1; ++k)
                    if (j < segs[k].size()) out.push_back(tl[segs[k][j]]);
        }
        r0 = r1;
    }
    tl.swap(out);
}

}  // namespace

struct gabor_batch_s {
    gabor_plan plan = nullptr;
    int32_t n = 0;
    std::vector<BatchImage> images;          // host copy (pointers, sizes)
    std::vector<BatchGroup> groups;          // fused launches, heaviest first
    std::vector<int> twopass_freqs;          // frequencies on the two-pass kernels
    BatchImage* d_images = nullptr;
    BatchFreq* d_freqs = nullptr;
    float2* d_J = nullptr;                   // J planes of the two-pass frequencies, every image
    int max_h = 0, max_w = 0;
    BatchTile* d_tiles = nullptr;
    int64_t tiles = 0;
};

namespace {

void batch_release(gabor_batch b)
{
    if (!b) return;
    if (b->d_images) (void)hipFree(b->d_images);
    if (b->d_freqs) (void)hipFree(b->d_freqs);
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    if (b->d_J) (void)hipFree(b->d_J);
    delete b;
}

}  // namespace

extern "C" gabor_status gabor_batch_create(gabor_batch* out, gabor_plan p, int32_t n_images,
                                           const float* const* d_images, const int32_t* heights,
                                           const int32_t* widths, const int64_t* row_strides,
                                           void* const* d_outs, void* hip_stream)
{
    if (!out) return GABOR_ERR_INVALID_ARG;
    *out = nullptr;
    if (!p || n_images <= 0 || !d_images || !heights || !widths || !row_strides || !d_outs)
        return GABOR_ERR_INVALID_ARG;
    if (p->iir) return GABOR_ERR_UNSUPPORTED;
    for (int i = 0; i < n_images; ++i) {
        if (!d_images[i] || !d_outs[i]) return GABOR_ERR_INVALID_ARG;
        if (heights[i] <= 0 || widths[i] <= 0 || heights[i] > p->H || widths[i] > p->W) return GABOR_ERR_INVALID_ARG;
        if (row_strides[i] < widths[i]) return GABOR_ERR_INVALID_ARG;
        if (!p->fjobs.empty() && (int64_t)(heights[i] - 1) * row_strides[i] + widths[i] >= (int64_t(1) << 30))
            return GABOR_ERR_UNSUPPORTED;
    }
    gabor_batch b = new (std::nothrow) gabor_batch_s;
    if (!b) return GABOR_ERR_OUT_OF_MEMORY;
    b->plan = p;
    b->n = n_images;
    const int sx = stream_strip_width();
    int64_t J_elems = 0;
    for (int i = 0; i < n_images; ++i) {
        BatchImage im{};
        im.J_off = J_elems;
        J_elems += (int64_t)p->n_planes * heights[i] * widths[i];
        b->max_h = std::max(b->max_h, (int)heights[i]);
        b->max_w = std::max(b->max_w, (int)widths[i]);
        im.img = d_images[i];
        im.out = (float2*)d_outs[i];
        im.stride = row_strides[i];
        im.H = heights[i];
        im.W = widths[i];
        im.n_xs = (widths[i] + sx - 1) / sx;
        b->images.push_back(im);
    }
    const std::vector<BatchFreq> freqs = batch_freq_table(p);
    for (int f = 0; f < p->O; ++f)
        if (!p->launches[f].fused) b->twopass_freqs.push_back(f);
    // One launch per quarter, or (plan option) one for every small quarter
    // of the wave-specialised kernel together (key 0) when there are several.
    auto small = [&](int q) { return p->group_small && p->use_ws && ws_small_quarter(p->fused_op, q); };
    std::vector<int> small_qs;
    for (int f = 0; f < p->O; ++f)
        if (p->launches[f].fused && small(p->launches[f].q) &&
            std::find(small_qs.begin(), small_qs.end(), p->launches[f].q) == small_qs.end())
            small_qs.push_back(p->launches[f].q);
    const bool merge = small_qs.size() > 1;
    auto key_of = [&](int f) { return merge && small(p->launches[f].q) ? 0 : p->launches[f].q; };
    // Tiles per launch: image-major, then segment, strip and job (jobs of a
    // strip share its image rows), then put in dispatch order (xcd_order).
    std::vector<int> qs;
    for (int f = 0; f < p->O; ++f)
        if (p->launches[f].fused && std::find(qs.begin(), qs.end(), key_of(f)) == qs.end())
            qs.push_back(key_of(f));
    std::vector<BatchTile> tiles;
    for (int key : qs) {
        BatchGroup g{};
        g.q = key;
        g.first_tile = (int)tiles.size();
        std::vector<std::pair<int64_t, BatchTile>> tl;    // (cost, tile)
        for (int i = 0; i < n_images; ++i)
            for (int f = 0; f < p->O; ++f) {
                const FreqLaunch& fl = p->launches[f];
                if (!fl.fused || key_of(f) != key) continue;
                const int q = fl.q;
                const int h = heights[i], seg = fl.seg_rows;
                const int n_ys = (h + seg - 1) / seg;
                const int lead = 4 * q / 16;
                for (int ys = 0; ys < n_ys; ++ys) {
                    const int steps = (std::min(seg, h - ys * seg) + 15) / 16 + lead;
                    for (int xs = 0; xs < b->images[i].n_xs; ++xs)
                        for (int j = 0; j < fl.count; ++j) {
                            // cost: steps times the products per step of the job
                            // kind (horizontal 2, or 1 for a real J; vertical 4,
                            // or 2 with a real J or real taps) plus a fixed
                            // per-step overhead
                            const FusedJob& jb = p->fjobs[fl.first + j];
                            const int per = q * ((jb.j_real ? 1 : 2) + (jb.j_real || jb.c_real ? 2 : 4)) + 16;
                            BatchTile t{};
                            t.image = i;
                            t.job = fl.first + j;
                            t.freq = f;
                            t.rest = xs + ys * b->images[i].n_xs;
                            tl.push_back({(int64_t)steps * per, t});
                            g.weight += (int64_t)steps * per;
                        }
                }
            }
        // profile name and algorithmic work: the group's frequencies over
        // every image, scaled from the plan's full-size figures
        {
            double macs = 0.0, bytes = 0.0;
            std::string radii;
            const double full = (double)p->H * p->W;
            for (int f = 0; f < p->O; ++f) {
                const FreqLaunch& fl = p->launches[f];
                if (!fl.fused || key_of(f) != key) continue;
                radii += (radii.empty() ? "" : "+") + std::to_string(p->freqs[f].R);
                for (int i = 0; i < n_images; ++i) {
                    const double frac = (double)heights[i] * widths[i] / full;
                    macs += (double)fl.macs * frac;
                    bytes += (double)fl.bytes * frac;
                }
            }
            const bool ws = key == 0 || (p->use_ws && ws_supported(p->fused_op, key));
            g.name = std::string(ws ? kWsNames[p->fused_op] : kFusedNames[p->fused_op]) + "_r" + radii +
                     (n_images > 1 ? "_x" + std::to_string(n_images) : std::string());
            g.macs = (int64_t)(macs + 0.5);
            g.bytes = (int64_t)(bytes + 0.5);
        }
        xcd_order(tl);
        if ((int64_t)tiles.size() + (int64_t)tl.size() > 0x7fffffffLL) {
            batch_release(b);
            return GABOR_ERR_UNSUPPORTED;
        }
        for (auto& e : tl) tiles.push_back(e.second);
        g.n_tiles = (int)tl.size();
        b->groups.push_back(g);
    }
    std::stable_sort(b->groups.begin(), b->groups.end(),
                     [](const BatchGroup& a, const BatchGroup& c) { return a.weight > c.weight; });
    b->tiles = (int64_t)tiles.size();

    hipStream_t stream = (hipStream_t)hip_stream;
    const size_t ib = b->images.size() * sizeof(BatchImage), fb = freqs.size() * sizeof(BatchFreq);
    const size_t tb = std::max<size_t>(1, tiles.size()) * sizeof(BatchTile);
    hipError_t e = hipMalloc((void**)&b->d_images, ib);
    if (e == hipSuccess && J_elems > 0) e = hipMalloc((void**)&b->d_J, (size_t)J_elems * sizeof(float2));
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_freqs, fb);
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_tiles, tb);
    if (e != hipSuccess) {
        batch_release(b);
        return e == hipErrorOutOfMemory ? GABOR_ERR_OUT_OF_MEMORY : GABOR_ERR_DEVICE;
    }
    if (hipMemcpyAsync(b->d_images, b->images.data(), ib, hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipMemcpyAsync(b->d_freqs, freqs.data(), fb, hipMemcpyHostToDevice, stream) != hipSuccess ||
        (!tiles.empty() &&
         hipMemcpyAsync(b->d_tiles, tiles.data(), tiles.size() * sizeof(BatchTile), hipMemcpyHostToDevice, stream) != hipSuccess) ||
        hipStreamSynchronize(stream) != hipSuccess) {
        batch_release(b);
        return GABOR_ERR_DEVICE;
    }
    *out = b;
    return GABOR_OK;
}

extern "C" gabor_status gabor_batch_apply(gabor_batch b, void* hip_stream)
{
    if (!b || !b->plan) return GABOR_ERR_INVALID_ARG;
    gabor_plan p = b->plan;
    hipStream_t stream = (hipStream_t)hip_stream;
    // Fork: launch j > 0 goes to auxiliary stream (j - 1) mod n after the
    // work already queued on the caller's stream.
    const int n_aux = (int)p->aux.size();
    const bool fork = n_aux > 0 && b->groups.size() > 1;
    if (fork) {
        if (hipEventRecord(p->fork_ev[0], stream) != hipSuccess) return GABOR_ERR_DEVICE;
        for (int k = 0; k < n_aux; ++k)
            if (hipStreamWaitEvent(p->aux[k], p->fork_ev[0], 0) != hipSuccess) return GABOR_ERR_DEVICE;
    }
    for (size_t j = 0; j < b->groups.size(); ++j) {
        const BatchGroup& g = b->groups[j];
        hipStream_t ls = (j == 0 || !fork) ? stream : p->aux[(j - 1) % n_aux];
        LaunchTimer tm(p, ls, g.name, g.macs, g.bytes);
        if (g.q == 0 || (p->use_ws && ws_supported(p->fused_op, g.q))) {
            // one workgroup per tile, tiles in decreasing cost
            WsTilesArgs t{};
            t.images = b->d_images;
            t.freqs = b->d_freqs;
            t.tiles = b->d_tiles + g.first_tile;
            t.jobs = p->d_fjobs;
            t.taps = p->d_taps;
            t.n_tiles = g.n_tiles;
            t.boundary = p->boundary;
            const hipError_t e = g.q == 0 ? launch_ws_tiles_small(p->fused_op, t, ls)
                                          : launch_ws_tiles(p->fused_op, t, g.q, ls);
            if (e != hipSuccess) return GABOR_ERR_DEVICE;
            continue;
        }
        BatchArgs a{};
        a.images = b->d_images;
        a.freqs = b->d_freqs;
        a.tiles = b->d_tiles + g.first_tile;
        a.jobs = p->d_fjobs;
        a.taps = p->d_taps;
        a.n_tiles = g.n_tiles;
        a.boundary = p->boundary;
        if (launch_batch(p->fused_op, a, g.q, ls) != hipSuccess) return GABOR_ERR_DEVICE;
    }
    // Two-pass frequencies: every image in one launch per horizontal group
    // and one per frequency (images in chunks that fit the grid), each image
    // with its own J planes.
    if (!b->twopass_freqs.empty()) {
        int max_jobs = 1;
        for (int f : b->twopass_freqs) max_jobs = std::max(max_jobs, p->launches[f].count);
        const int chunk = std::max(1, std::min(65535, 65535 / max_jobs));
        for (int i0 = 0; i0 < b->n; i0 += chunk) {
            const int n = std::min(chunk, b->n - i0);
            for (size_t gi = 0; gi < p->row_groups.size(); ++gi) {
                const RowGroup& rg = p->row_groups[gi];
                if (launch_row_fp32_batch(b->d_images + i0, n, b->max_h, b->max_w, p->boundary, p->freqs[rg.freq], rg,
                                          p->d_taps, b->d_J, stream) != hipSuccess)
                    return GABOR_ERR_DEVICE;
            }
            for (int f : b->twopass_freqs) {
                const FreqLaunch& fl = p->launches[f];
                if (launch_col_fp32_batch(b->d_images + i0, n, b->max_h, b->max_w, p->boundary, p->freqs[f],
                                          p->d_jobs + fl.first, fl.count, p->d_taps, b->d_J, stream) != hipSuccess)
                    return GABOR_ERR_DEVICE;
            }
        }
    }
    if (fork) {
        for (int k = 0; k < n_aux; ++k)
            if (hipEventRecord(p->join_ev[k], p->aux[k]) != hipSuccess ||
                hipStreamWaitEvent(stream, p->join_ev[k], 0) != hipSuccess)
                return GABOR_ERR_DEVICE;
    }
    return GABOR_OK;
}

extern "C" gabor_status gabor_batch_info(gabor_batch b, int32_t* n_launches, int64_t* n_tiles)
{
    if (!b) return GABOR_ERR_INVALID_ARG;
    if (n_launches) *n_launches = (int32_t)b->groups.size();
    if (n_tiles) *n_tiles = b->tiles;
    return GABOR_OK;
}

extern "C" gabor_status gabor_batch_destroy(gabor_batch b)
{
    batch_release(b);
    return GABOR_OK;
}
