// Host side of libhs: plan creation (shape checks, candidate-word widths,
// tile geometry), argument validation and kernel dispatch.  Every entry point
// returns an hs_status and catches C++ exceptions before they reach the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "hs_internal.h"

namespace hsk {
// SingleHP baseline (hs_singlehp.hip)
hipError_t launch_singlehp(const float* fop, int64_t ld, int T, int N, int H, const float* ta, hs_cand* out,
                           int64_t cap, unsigned long long* counts, int s_row, int s_bin, float* work,
                           bool single_launch, hipStream_t s);
// Per-plane capped lists (hs_select.hip)
hipError_t select_workspace(int64_t n, int end_bit, size_t* bytes);
hipError_t select_top(const uint64_t* cand, int64_t n, int H, int s_bin, int s_k, int n_cand, uint64_t* out,
                      int64_t* out_counts, void* work, hipStream_t s);
}  // namespace hsk

namespace {

int ceil_log2(int64_t x)
{
    int s = 0;
    while (((int64_t)1 << s) < x) ++s;
    return s;
}

bool is_pow2_scale(float s)
{
    if (!(s > 0.0f) || !std::isfinite(s)) return false;
    int e = 0;
    return std::frexp(s, &e) == 0.5f;
}

int elem_bytes(int dtype) { return dtype == HS_DTYPE_F32 ? 4 : 2; }
int ld_align(int dtype) { return dtype == HS_DTYPE_F32 ? 4 : 8; }

// Largest LDS footprint the planner gives one block, so that two blocks fit
// in the 160 KiB of a gfx950 compute unit.
constexpr int kLdsBudget = 80 * 1024;

hs_status from_hip(hipError_t e) { return e == hipSuccess ? HS_OK : HS_ERR_HIP; }

bool fop_ok(const hs_plan* p, const void* fop, int64_t ld, int64_t N)
{
    if (!fop || ld < N) return false;
    if (reinterpret_cast<uintptr_t>(fop) & 15) return false;
    // the staging addresses source words by 32-bit byte offsets within the
    // source rows of one stretch factor (at most stage_rows(2) rows)
    if ((ld * hsk::stage_rows(2) + hsk::kTileBins) * elem_bytes(p->dtype) >= ((int64_t)1 << 32))
        return false;
    return ld % ld_align(p->dtype) == 0;
}

// Full-tile schedule of a single-FOP plan (the kernel side is described in
// hs_fused_impl.h).  Bin tile x >= 8 lies in octave L = floor(log2 x); list
// k holds the tiles whose bits L-1..L-3 equal k (tiles 0..7 go to list x),
// ordered by their position inside that sub-range scaled to the top octave,
// then by L (so x/2, x/4, x/8 come just before x), then by row block.
// Layout: nine list offsets, then the entries (rb << 24) | x.  Empty when
// the fields do not fit.
std::vector<uint32_t> build_schedule(int64_t n_full, int row_blocks)
{
    std::vector<uint32_t> out;
    if (n_full < 1 || row_blocks < 1 || row_blocks > 255 || n_full >= ((int64_t)1 << 24)) return out;
    int top = 0;
    while (((int64_t)2 << top) <= n_full - 1) ++top;      // floor(log2(n_full - 1)), 0 for n_full <= 2
    struct E { int64_t key; int L; int64_t x; };
    std::vector<E> lists[8];
    for (int64_t x = 0; x < n_full; ++x) {
        if (x < 8) {
            lists[x].push_back({0, -1, x});
            continue;
        }
        int L = 3;
        while (((int64_t)2 << L) <= x) ++L;
        const int64_t off = x - ((int64_t)1 << L);
        const int k = (int)(off >> (L - 3));
        const int64_t pos = off & (((int64_t)1 << (L - 3)) - 1);
        lists[k].push_back({pos << (top - L), L, x});
    }
    out.assign(9, 0);
    for (int k = 0; k < 8; ++k) {
        std::sort(lists[k].begin(), lists[k].end(), [](const E& a, const E& b) {
            if (a.key != b.key) return a.key < b.key;
            if (a.L != b.L) return a.L < b.L;
            return a.x < b.x;
        });
        out[k + 1] = out[k] + (uint32_t)(lists[k].size() * row_blocks);
    }
    for (int k = 0; k < 8; ++k)
        for (const E& e : lists[k])
            for (int rb = 0; rb < row_blocks; ++rb) out.push_back(((uint32_t)rb << 24) | (uint32_t)e.x);
    return out;
}

// Strip order of the walk kernel for one FOP of n_strips strips of 256 bins
// (the kernel side is described in hs_walk_impl.h).  Strip x >= 8 lies in
// octave L = floor(log2 x) at position (x - 2^L) / 2^L; its list is the three
// bits after the leading one, and dividing x by 2, 4 or 8 keeps both the list
// and the position scaled to the top octave.  Strips are ordered by that
// position, then by octave (x/8, x/4, x/2 just before x), then by index.
// lists == 8: one list per XCD; lists == 1: one list of all strips.
std::vector<std::vector<uint32_t>> walk_strip_lists(int64_t n_strips, int lists, bool linear = false)
{
    std::vector<std::vector<uint32_t>> out(lists);
    if (n_strips < 1) return out;
    if (linear) {
        // increasing strip order, dealt to the lists in turn
        for (int64_t x = 0; x < n_strips; ++x) out[x % lists].push_back((uint32_t)x);
        return out;
    }
    int top = 0;
    while (((int64_t)2 << top) <= n_strips - 1) ++top;
    struct E { int64_t key; int L; int64_t x; };
    std::vector<E> l[8];
    for (int64_t x = 0; x < n_strips; ++x) {
        if (x < 8) {
            l[lists == 8 ? x : 0].push_back({0, -1, x});
            continue;
        }
        int L = 3;
        while (((int64_t)2 << L) <= x) ++L;
        const int64_t off = x - ((int64_t)1 << L);
        const int k = (int)(off >> (L - 3));
        const int64_t pos = off & (((int64_t)1 << (L - 3)) - 1);
        l[lists == 8 ? k : 0].push_back({(pos << (top - L)) << 3 | k, L, x});
    }
    for (int k = 0; k < lists; ++k) {
        std::sort(l[k].begin(), l[k].end(), [](const E& a, const E& b) {
            if (a.key != b.key) return a.key < b.key;
            if (a.L != b.L) return a.L < b.L;
            return a.x < b.x;
        });
        for (const E& e : l[k]) out[k].push_back((uint32_t)e.x);
    }
    return out;
}

// Walk tables of a plan: units (band << 24) | strip for every band of every
// strip; a single FOP spreads its strips over eight XCD lists, a batch puts
// each FOP whole on one XCD (longest first onto the least loaded XCD).
// Device layout: xseg [9] u32 | rowmask [T] u32 | seg [n_seg][4] i32 |
// n_chans [n_fops] i64 | entries u32.
void build_walk(hs_plan* p, bool linear)
{
    const int T = (int)p->T;
    const int c = T / 2;
    // the two half-planes as bands when each has at least kWalkDepth rows
    // (the kernel keeps that many rows in flight and starts at most one unit
    // inside them), else the full height as one band
    p->band_split = (c >= hsk::kWalkDepth && T - c >= hsk::kWalkDepth) ? c : 0;
    const int bands = p->band_split > 0 ? 2 : 1;
    std::vector<uint32_t> rowmask(T, 0u);
    for (int r = 0; r < T; ++r)
        for (int m = 2; m <= hsk::kMaxH; ++m)
            if (((r - c) % m + m) % m == 0) rowmask[r] |= 1u << m;

    std::vector<uint32_t> ent;
    std::vector<int32_t> seg;   // 4 per segment
    std::vector<uint32_t> xseg(9, 0);
    auto add_units = [&](const std::vector<uint32_t>& strips) {
        const size_t first = ent.size();
        for (int b = 0; b < bands; ++b)
            for (uint32_t x : strips) ent.push_back(((uint32_t)b << 24) | x);
        return std::make_pair((int64_t)first, (int64_t)(ent.size() - first));
    };
    std::vector<int64_t> nchan;
    if (p->n_fops == 0) {
        const int64_t sb = 64 * (int64_t)p->walk_v;
        const auto lists = walk_strip_lists((p->N + sb - 1) / sb, 8, linear);
        for (int x = 0; x < 8; ++x) {
            xseg[x] = (uint32_t)(seg.size() / 4);
            const auto r = add_units(lists[x]);
            if (r.second > 0) {
                seg.insert(seg.end(), {0, (int32_t)r.first, 0, (int32_t)r.second});
            }
        }
        xseg[8] = (uint32_t)(seg.size() / 4);
    } else {
        // one unit list per distinct length
        std::vector<std::pair<int64_t, std::pair<int64_t, int64_t>>> by_len;   // N -> (first, count)
        std::vector<std::pair<int64_t, int64_t>> fl(p->n_fops);
        for (int f = 0; f < p->n_fops; ++f) {
            const int64_t n = p->n_chans[f];
            auto it = std::find_if(by_len.begin(), by_len.end(), [&](const auto& e) { return e.first == n; });
            if (it == by_len.end()) {
                const int64_t sb = 64 * (int64_t)p->walk_v;
                const auto lists = walk_strip_lists((n + sb - 1) / sb, 1, linear);
                by_len.push_back({n, add_units(lists[0])});
                it = by_len.end() - 1;
            }
            fl[f] = it->second;
        }
        // whole FOPs to XCDs: longest first onto the least loaded
        std::vector<int> order(p->n_fops);
        for (int f = 0; f < p->n_fops; ++f) order[f] = f;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return fl[a].second > fl[b].second; });
        std::vector<std::vector<int>> on(8);
        int64_t load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int f : order) {
            int best = 0;
            for (int x = 1; x < 8; ++x)
                if (load[x] < load[best]) best = x;
            on[best].push_back(f);
            load[best] += fl[f].second;
        }
        for (int x = 0; x < 8; ++x) {
            std::sort(on[x].begin(), on[x].end());
            xseg[x] = (uint32_t)(seg.size() / 4);
            int64_t pre = 0;
            for (int f : on[x]) {
                if (fl[f].second == 0) continue;
                seg.insert(seg.end(), {(int32_t)f, (int32_t)fl[f].first, (int32_t)pre, (int32_t)(pre + fl[f].second)});
                pre += fl[f].second;
            }
        }
        xseg[8] = (uint32_t)(seg.size() / 4);
        nchan = p->n_chans;
    }

    auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
    p->off_xseg = 0;
    p->off_rowmask = align(p->off_xseg + xseg.size() * 4);
    p->off_seg = align(p->off_rowmask + rowmask.size() * 4);
    p->off_nchan = align(p->off_seg + seg.size() * 4);
    p->off_ent = align(p->off_nchan + nchan.size() * 8);
    p->walk_tab.assign(align(p->off_ent + ent.size() * 4), 0);
    std::memcpy(p->walk_tab.data() + p->off_xseg, xseg.data(), xseg.size() * 4);
    std::memcpy(p->walk_tab.data() + p->off_rowmask, rowmask.data(), rowmask.size() * 4);
    if (!seg.empty()) std::memcpy(p->walk_tab.data() + p->off_seg, seg.data(), seg.size() * 4);
    if (!nchan.empty()) std::memcpy(p->walk_tab.data() + p->off_nchan, nchan.data(), nchan.size() * 8);
    if (!ent.empty()) std::memcpy(p->walk_tab.data() + p->off_ent, ent.data(), ent.size() * 4);
    p->walk_lds = hsk::walk_lds_bytes(T, p->H, p->dtype, p->walk_v);
    p->walk = true;
}

// Device copies of a plan's tables on one device.
struct DevTabs {
    const unsigned char* walk = nullptr;   // strip-walk units and row table
    const uint32_t* sched = nullptr;       // full-tile schedule (null: contiguous chunks)
    const int64_t* batch = nullptr;        // batched: bins of each FOP, then the tile prefix
};

hs_status copy_to_device(const void* src, size_t bytes, void** dst)
{
    void* d = nullptr;
    if (hipMalloc(&d, bytes) != hipSuccess) return HS_ERR_NOMEM;
    if (hipMemcpy(d, src, bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d);
        return HS_ERR_HIP;
    }
    *dst = d;
    return HS_OK;
}

// Every table the plan has, on the current device: all are copied together
// (synchronously) by the first call on a device that is not under stream
// capture, or by hs_plan_upload.  A call under capture on a device that has
// no copy yet gets HS_ERR_INVALID, since a copy cannot be made inside a
// graph; so does a stream of another device than the current one (the
// tables are per device).
hs_status device_tables(const hs_plan* p, hipStream_t stream, DevTabs* t)
{
    *t = DevTabs{};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return HS_ERR_HIP;
    if (stream) {
        hipDevice_t sd = 0;
        if (hipStreamGetDevice(stream, &sd) != hipSuccess || (int)sd != dev) return HS_ERR_INVALID;
    }
    std::lock_guard<std::mutex> g(p->mu);
    const bool need_walk = p->walk && !p->d_walk[dev];
    const bool need_sched = !p->sched.empty() && !p->d_sched[dev];
    const bool need_batch = p->n_fops > 0 && !p->d_tables[dev];
    if (need_walk || need_sched || need_batch) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(stream, &cs) != hipSuccess) return HS_ERR_HIP;
        if (cs != hipStreamCaptureStatusNone) return HS_ERR_INVALID;
        void* d = nullptr;
        if (need_walk) {
            const hs_status st = copy_to_device(p->walk_tab.data(), p->walk_tab.size(), &d);
            if (st != HS_OK) return st;
            p->d_walk[dev] = static_cast<unsigned char*>(d);
        }
        if (need_sched) {
            const hs_status st = copy_to_device(p->sched.data(), p->sched.size() * sizeof(uint32_t), &d);
            if (st != HS_OK) return st;
            p->d_sched[dev] = static_cast<uint32_t*>(d);
        }
        if (need_batch) {
            std::vector<int64_t> h((size_t)p->n_fops * 2 + 1);
            for (int f = 0; f < p->n_fops; ++f) h[f] = p->n_chans[f];
            for (int f = 0; f <= p->n_fops; ++f) h[p->n_fops + f] = p->tile_prefix[f];
            const hs_status st = copy_to_device(h.data(), h.size() * sizeof(int64_t), &d);
            if (st != HS_OK) return st;
            p->d_tables[dev] = static_cast<int64_t*>(d);
        }
    }
    t->walk = p->d_walk[dev];
    t->sched = p->d_sched[dev];
    t->batch = p->d_tables[dev];
    return HS_OK;
}

// The tables already on the current device, copying nothing (what is not
// there yet is null: the tile kernels then take contiguous chunks, with the
// same results).  HS_ERR_INVALID for a stream of another device.
hs_status device_tables_present(const hs_plan* p, hipStream_t stream, DevTabs* t)
{
    *t = DevTabs{};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return HS_ERR_HIP;
    if (stream) {
        hipDevice_t sd = 0;
        if (hipStreamGetDevice(stream, &sd) != hipSuccess || (int)sd != dev) return HS_ERR_INVALID;
    }
    std::lock_guard<std::mutex> g(p->mu);
    t->walk = p->d_walk[dev];
    t->sched = p->d_sched[dev];
    t->batch = p->d_tables[dev];
    return HS_OK;
}

hsk::WalkArgs walk_args(const hs_plan* p, const unsigned char* tab)
{
    hsk::WalkArgs a{};
    a.T = (int32_t)p->T;
    a.c = (int32_t)(p->T / 2);
    a.band_split = p->band_split;
    a.scale = p->scale;
    a.inv_scale = 1.0f / p->scale;
    a.s_row = p->s_row;
    a.s_bin = p->s_bin;
    a.xseg = reinterpret_cast<const uint32_t*>(tab + p->off_xseg);
    a.rowmask = reinterpret_cast<const uint32_t*>(tab + p->off_rowmask);
    a.seg = reinterpret_cast<const int32_t*>(tab + p->off_seg);
    a.n_chans = reinterpret_cast<const int64_t*>(tab + p->off_nchan);
    a.ent = reinterpret_cast<const uint32_t*>(tab + p->off_ent);
    return a;
}

hsk::FracArgs frac_args(const hs_plan* p, const void* fop, int64_t ld)
{
    hsk::FracArgs a{};
    a.fop = fop;
    a.ld = ld;
    a.T = (int32_t)p->T;
    a.c = (int32_t)(p->T / 2);
    a.N = (int32_t)p->N;
    a.H = p->H;
    a.scale = p->scale;
    a.inv_scale = 1.0f / p->scale;
    a.s_row = p->s_row;
    a.s_bin = p->s_bin;
    hsk::frac_magic(a);
    return a;
}

hsk::TileArgs tile_args(const hs_plan* p, const void* fop, int64_t ld, const DevTabs& t)
{
    hsk::TileArgs a{};
    a.fop = fop;
    a.ld = ld;
    a.N = p->N;
    a.T = (int32_t)p->T;
    a.c = (int32_t)(p->T / 2);
    a.R = p->tile_rows;
    a.row_blocks = p->row_blocks;
    a.scale = p->scale;
    a.inv_scale = 1.0f / p->scale;
    a.s_row = p->s_row;
    a.s_bin = p->s_bin;
    a.kmask = (1u << p->s_k) - 1u;
    a.table_whole = hsk::table_whole((int)p->T, p->H) ? 1 : 0;
    a.sched = t.sched;
    return a;
}

int64_t bin_tiles(int64_t n) { return (n + hsk::kTileBins - 1) / hsk::kTileBins; }

// Persistent grid override (0: the launcher sizes the grid from occupancy).
int persistent_grid(const hs_plan* p, int64_t tiles)
{
    (void)tiles;
    return p->persistent_blocks;
}

}  // namespace

extern "C" {

hs_status hs_plan_create(hs_plan** out, const hs_plan_desc* d)
{
    if (!out || !d) return HS_ERR_INVALID;
    *out = nullptr;
    try {
        if (d->n_temp < 1 || d->n_temp > (1 << 20)) return HS_ERR_INVALID;
        if (d->n_hp < 1 || d->n_hp > hsk::kMaxH) return HS_ERR_INVALID;
        if (d->dtype != HS_DTYPE_F32 && d->dtype != HS_DTYPE_F16 && d->dtype != HS_DTYPE_BF16)
            return HS_ERR_INVALID;
        const float scale = d->input_scale == 0.0f ? 1.0f : d->input_scale;
        if (!is_pow2_scale(scale)) return HS_ERR_INVALID;
        if (d->dtype == HS_DTYPE_F32 && scale != 1.0f) return HS_ERR_INVALID;
        if (d->n_fops < 0 || d->n_fops > 65535) return HS_ERR_INVALID;
        if (d->tile_rows < 0 || d->persistent_blocks < 0) return HS_ERR_INVALID;
        if (d->schedule < 0 || d->schedule > 4) return HS_ERR_INVALID;
        if (d->mapping != HS_MAP_PAPER && d->mapping != HS_MAP_FRACTIONAL) return HS_ERR_INVALID;
        if (d->bins_per_lane != 0 && !hsk::walk_v_ok(d->bins_per_lane)) return HS_ERR_INVALID;
        if (d->mapping == HS_MAP_FRACTIONAL && (d->n_fops != 0 || d->n_chan > hsk::kFracMaxBins))
            return HS_ERR_INVALID;

        hs_plan* p = new hs_plan();
        p->mapping = d->mapping;
        // bins per lane of the strip walk: eight for 16-bit storage up to
        // eight planes (the rings of 512-bin strips still leave four waves
        // per SIMD) and for batches (measured faster at H = 16, fp32), else
        // four
        p->walk_v = d->bins_per_lane ? d->bins_per_lane
                                     : ((d->dtype != HS_DTYPE_F32 && d->n_hp <= 8) || d->n_fops > 0 ? 8 : 4);
        p->T = d->n_temp;
        p->H = d->n_hp;
        p->dtype = d->dtype;
        p->scale = scale;
        p->n_fops = d->n_fops;
        p->persistent_blocks = d->persistent_blocks;
        int64_t nmax = 0;
        if (d->n_fops == 0) {
            if (d->n_chan < 1 || d->n_chan > INT32_MAX) { delete p; return HS_ERR_INVALID; }
            nmax = d->n_chan;
        } else {
            if (!d->n_chans) { delete p; return HS_ERR_INVALID; }
            p->n_chans.assign(d->n_chans, d->n_chans + d->n_fops);
            for (int64_t n : p->n_chans) {
                if (n < 1 || n > INT32_MAX) { delete p; return HS_ERR_INVALID; }
                if (n > nmax) nmax = n;
            }
        }
        p->N = nmax;
        p->s_bin = ceil_log2(nmax);
        p->s_k = ceil_log2(p->H);
        const int s_r = ceil_log2(p->T);
        if (p->s_bin + p->s_k + s_r > 32) { delete p; return HS_ERR_INVALID; }
        p->s_row = p->s_bin + p->s_k;

        // Rows per tile: kMaxTileRows (the staging layout is sized for it;
        // the last row block may be shorter), or fewer on request.
        int R = (int)std::min<int64_t>(d->tile_rows > 0 ? d->tile_rows : hsk::kMaxTileRows, p->T);
        if (R > hsk::kMaxTileRows ||
            hsk::fused_lds_bytes((int)p->T, R, p->H, hsk::kModeDetect, elem_bytes(p->dtype)) > kLdsBudget) {
            delete p;
            return HS_ERR_UNSUPPORTED;
        }
        p->tile_rows = R;
        p->row_blocks = (int)((p->T + R - 1) / R);
        p->lds_bytes = hsk::fused_lds_bytes((int)p->T, R, p->H, hsk::kModeDetect, elem_bytes(p->dtype));

        // detection: the strip walk (XCD lists by octave position; increasing
        // strip order for schedule 1) where its threshold table fits and it
        // is the faster kernel, else the tile kernel.  Measured on 85 x 2^21
        // planes, the walk wins with 16-bit storage and with more than eight
        // planes, the tile kernel with fp32 storage up to eight: schedule 0
        // picks by that rule, 1 and 4 ask for the walk, 2 and 3 for the tile
        // kernel.  The tile kernels of the other calls use the XCD tile
        // schedule for 0, 2 and 4, contiguous chunks for 1 and 3.
        const bool walk_wins = p->dtype != HS_DTYPE_F32 || p->H > 8;
        const bool want_walk = d->schedule == 1 || d->schedule == 4 || (d->schedule == 0 && walk_wins);
        const bool paper = d->mapping == HS_MAP_PAPER;   // the fractional mapping has a kernel of its own
        if (paper && want_walk && hsk::walk_supported((int)p->T, p->H)) build_walk(p, d->schedule == 1);

        if (d->n_fops == 0) {
            p->tiles_total = p->row_blocks * bin_tiles(p->N);
            if (paper && (d->schedule == 0 || d->schedule == 2 || d->schedule == 4))
                p->sched = build_schedule(p->N / hsk::kTileBins, p->row_blocks);
        } else {
            p->tile_prefix.resize(d->n_fops + 1);
            int64_t acc = 0;
            for (int f = 0; f < d->n_fops; ++f) {
                p->tile_prefix[f] = acc;
                acc += p->row_blocks * bin_tiles(p->n_chans[f]);
            }
            p->tile_prefix[d->n_fops] = acc;
            p->tiles_total = acc;
        }
        *out = p;
        return HS_OK;
    } catch (const std::bad_alloc&) {
        return HS_ERR_NOMEM;
    } catch (...) {
        return HS_ERR_INVALID;
    }
}

hs_status hs_plan_destroy(hs_plan* p)
{
    if (!p) return HS_OK;
    int cur = -1;
    bool have_dev = hipGetDevice(&cur) == hipSuccess;
    for (int dev = 0; dev < 64; ++dev) {
        if (p->d_tables[dev] || p->d_sched[dev] || p->d_walk[dev]) {
            if (have_dev) (void)hipSetDevice(dev);
            if (p->d_tables[dev]) (void)hipFree(p->d_tables[dev]);
            if (p->d_sched[dev]) (void)hipFree(p->d_sched[dev]);
            if (p->d_walk[dev]) (void)hipFree(p->d_walk[dev]);
        }
    }
    if (have_dev && cur >= 0) (void)hipSetDevice(cur);
    delete p;
    return HS_OK;
}

int64_t hs_plan_schedule(const hs_plan* p, uint32_t* words, int64_t capacity)
{
    if (!p) return -1;
    const int64_t n = (int64_t)p->sched.size();
    if (words && capacity > 0) std::memcpy(words, p->sched.data(), (size_t)std::min(n, capacity) * 4);
    return n;
}

hs_status hs_plan_upload(const hs_plan* p)
{
    if (!p) return HS_ERR_INVALID;
    try {
        DevTabs t;
        return device_tables(p, nullptr, &t);
    } catch (...) {
        return HS_ERR_HIP;
    }
}

hs_status hs_plan_info_get(const hs_plan* p, hs_plan_info* info)
{
    if (!p || !info) return HS_ERR_INVALID;
    std::memset(info, 0, sizeof(*info));
    info->n_temp = (int32_t)p->T;
    info->n_hp = p->H;
    info->dtype = p->dtype;
    info->n_fops = p->n_fops;
    info->n_chan_max = p->N;
    info->s_row = p->s_row;
    info->s_k = p->s_k;
    info->s_bin = p->s_bin;
    info->tile_bins = hsk::kTileBins;
    info->tile_rows = p->tile_rows;
    info->row_blocks = p->row_blocks;
    info->lds_bytes = p->lds_bytes;
    info->tiles_total = p->tiles_total;
    info->detector = p->mapping == HS_MAP_FRACTIONAL ? 2 : (p->walk ? 1 : 0);
    info->mapping = p->mapping;
    info->bins_per_lane = p->walk ? p->walk_v : 0;
    // distinct source rows of each stretch factor over the full column, and the
    // words one full-height tile at a 256-bin aligned position stages
    const int64_t c = p->T / 2;
    int64_t staged = 0;
    for (int m = 1; m <= p->H; ++m) {
        const int64_t rows = hsk::floordiv(p->T - 1 - c, m) - hsk::floordiv(-c, m) + 1;
        info->src_rows[m] = (int32_t)rows;
        if (m >= 2) staged += rows * ((hsk::kTileBins - 1) / m + 1);
    }
    info->staged_words = staged;
    return HS_OK;
}

hs_status hs_sum(const hs_plan* p, const void* fop, int64_t ld, float* hp, void* stream)
{
    if (!p || !hp || p->n_fops != 0) return HS_ERR_INVALID;
    if (!fop_ok(p, fop, ld, p->N)) return HS_ERR_INVALID;
    try {
        if (p->mapping == HS_MAP_FRACTIONAL) {
            hsk::FracArgs a = frac_args(p, fop, ld);
            a.hp = hp;
            return from_hip(hsk::launch_frac(p->dtype, false, a, (hipStream_t)stream));
        }
        DevTabs t;
        const hs_status st = device_tables(p, (hipStream_t)stream, &t);
        if (st != HS_OK) return st;
        hsk::TileArgs a = tile_args(p, fop, ld, t);
        a.hp = hp;
        return from_hip(hsk::launch_fused(hsk::kModeSum, p->dtype, p->H, a, p->tiles_total,
                                          persistent_grid(p, p->tiles_total), p->lds_bytes,
                                          (hipStream_t)stream));
    } catch (...) {
        return HS_ERR_HIP;
    }
}

hs_status hs_detect(const hs_plan* p, const void* fop, int64_t ld, const float* ta, hs_cand* out,
                    int64_t capacity, int64_t* counts, void* stream)
{
    if (!p || p->n_fops != 0 || !ta || !counts || capacity < 0) return HS_ERR_INVALID;
    if (capacity > 0 && !out) return HS_ERR_INVALID;
    if (!fop_ok(p, fop, ld, p->N)) return HS_ERR_INVALID;
    try {
        hipStream_t s = (hipStream_t)stream;
        DevTabs t;
        const hs_status st = device_tables(p, s, &t);
        if (st != HS_OK) return st;
        if (p->mapping == HS_MAP_FRACTIONAL) {
            if (hsk::launch_zero_i64(counts, p->H + 1, s) != hipSuccess) return HS_ERR_HIP;
            hsk::FracArgs a = frac_args(p, fop, ld);
            a.ta = ta;
            a.out = out;
            a.cap = capacity;
            a.counts = reinterpret_cast<unsigned long long*>(counts);
            if (hsk::launch_frac(p->dtype, true, a, s) != hipSuccess) return HS_ERR_HIP;
        } else if (p->walk) {
            if (hsk::launch_zero_i64(counts, p->H + 1, s) != hipSuccess) return HS_ERR_HIP;
            hsk::WalkArgs a = walk_args(p, t.walk);
            a.fop = fop;
            a.ld = ld;
            a.N = (int32_t)p->N;
            a.n_fops = 0;
            a.ta = ta;
            a.out = out;
            a.cap = capacity;
            a.counts = reinterpret_cast<unsigned long long*>(counts);
            if (hsk::launch_walk(p->dtype, p->H, p->walk_v, a, p->persistent_blocks, p->walk_lds, s) != hipSuccess)
                return HS_ERR_HIP;
        } else {
            hipError_t e = hsk::launch_zero_i64(counts, p->H + 1, s);
            if (e != hipSuccess) return HS_ERR_HIP;
            hsk::TileArgs a = tile_args(p, fop, ld, t);
            a.ta = ta;
            a.out = out;
            a.cap = capacity;
            a.counts = reinterpret_cast<unsigned long long*>(counts);
            if (hsk::launch_fused(hsk::kModeDetect, p->dtype, p->H, a, p->tiles_total,
                                  persistent_grid(p, p->tiles_total), p->lds_bytes, s) != hipSuccess)
                return HS_ERR_HIP;
        }
        if (capacity == 0) return HS_OK;
        return from_hip(hsk::launch_plane_counts(out, nullptr, nullptr, capacity,
                                                 reinterpret_cast<unsigned long long*>(counts), 1, p->H,
                                                 p->s_bin, (1u << p->s_k) - 1u, s));
    } catch (...) {
        return HS_ERR_HIP;
    }
}

size_t hs_select_workspace_bytes(const hs_plan* p, int64_t n)
{
    if (!p || n < 0) return 0;
    size_t bytes = 0;
    if (hsk::select_workspace(n, 32 + p->s_k, &bytes) != hipSuccess) return 0;
    return std::max(bytes, hsk::select_bounded_workspace(n, p->H, hsk::kSelLdsCand));
}

hs_status hs_select(const hs_plan* p, const hs_cand* cand, int64_t n, int32_t n_cand, int32_t policy, hs_cand* out,
                    int64_t* out_counts, void* work, void* stream)
{
    if (!p || n < 0 || n_cand < 1 || !out || !out_counts || !work) return HS_ERR_INVALID;
    if (policy != HS_SELECT_TOP && policy != HS_SELECT_LAST_ALG2 && policy != HS_SELECT_LAST_ALG1)
        return HS_ERR_INVALID;
    if (n > 0 && !cand) return HS_ERR_INVALID;
    try {
        const uint64_t* c = reinterpret_cast<const uint64_t*>(cand);
        uint64_t* o = reinterpret_cast<uint64_t*>(out);
        hipStream_t s = (hipStream_t)stream;
        if (n_cand <= hsk::kSelLdsCand && n <= (int64_t)UINT32_MAX)
            return from_hip(hsk::select_bounded(c, n, p->H, p->s_bin, p->s_k, policy, n_cand, o, out_counts, work, s));
        if (policy != HS_SELECT_TOP) return HS_ERR_UNSUPPORTED;
        return from_hip(hsk::select_top(c, n, p->H, p->s_bin, p->s_k, n_cand, o, out_counts, work, s));
    } catch (...) {
        return HS_ERR_HIP;
    }
}

hs_status hs_select_top(const hs_plan* p, const hs_cand* cand, int64_t n, int32_t n_cand, hs_cand* out,
                        int64_t* out_counts, void* work, void* stream)
{
    return hs_select(p, cand, n, n_cand, HS_SELECT_TOP, out, out_counts, work, stream);
}

size_t hs_singlehp_workspace_bytes(const hs_plan* p)
{
    if (!p || p->n_fops != 0 || p->dtype != HS_DTYPE_F32) return 0;
    return 2 * (size_t)((p->T * p->N + 63) & ~(int64_t)63) * sizeof(float);
}

namespace {

hs_status singlehp(const hs_plan* p, const float* fop, int64_t ld, const float* ta, hs_cand* out, int64_t capacity,
                   int64_t* counts, void* work, bool single_launch, void* stream)
{
    if (!p || p->n_fops != 0 || !ta || !counts || !work || capacity < 0) return HS_ERR_INVALID;
    if (p->dtype != HS_DTYPE_F32 || p->mapping != HS_MAP_PAPER) return HS_ERR_UNSUPPORTED;
    if (capacity > 0 && !out) return HS_ERR_INVALID;
    if (!fop_ok(p, fop, ld, p->N)) return HS_ERR_INVALID;
    try {
        hipStream_t s = (hipStream_t)stream;
        hipError_t e = hsk::launch_zero_i64(counts, p->H + 1, s);
        if (e != hipSuccess) return HS_ERR_HIP;
        return from_hip(hsk::launch_singlehp(fop, ld, (int)p->T, (int)p->N, p->H, ta, out, capacity,
                                             reinterpret_cast<unsigned long long*>(counts), p->s_row, p->s_bin,
                                             static_cast<float*>(work), single_launch, s));
    } catch (...) {
        return HS_ERR_HIP;
    }
}

}  // namespace

hs_status hs_detect_singlehp(const hs_plan* p, const float* fop, int64_t ld, const float* ta, hs_cand* out,
                             int64_t capacity, int64_t* counts, void* work, void* stream)
{
    return singlehp(p, fop, ld, ta, out, capacity, counts, work, false, stream);
}

hs_status hs_detect_singlehp_one(const hs_plan* p, const float* fop, int64_t ld, const float* ta, hs_cand* out,
                                 int64_t capacity, int64_t* counts, void* work, void* stream)
{
    return singlehp(p, fop, ld, ta, out, capacity, counts, work, true, stream);
}

hs_status hs_detect_batched(const hs_plan* p, const void* const* fops, const int64_t* lds,
                            const float* ta, hs_cand* out, const int64_t* out_offsets,
                            const int64_t* caps, int64_t* counts, void* stream)
{
    if (!p || p->n_fops < 1 || !fops || !lds || !ta || !out || !out_offsets || !caps || !counts)
        return HS_ERR_INVALID;
    try {
        hipStream_t s = (hipStream_t)stream;
        DevTabs t;
        const hs_status st = device_tables(p, s, &t);
        if (st != HS_OK) return st;
        if (p->walk) {
            if (hsk::launch_zero_i64(counts, (int64_t)p->n_fops * (p->H + 1), s) != hipSuccess) return HS_ERR_HIP;
            hsk::WalkArgs a = walk_args(p, t.walk);
            a.n_fops = p->n_fops;
            a.fops = fops;
            a.lds = lds;
            a.out_offsets = out_offsets;
            a.caps = caps;
            a.ta = ta;
            a.out = out;
            a.counts = reinterpret_cast<unsigned long long*>(counts);
            if (hsk::launch_walk(p->dtype, p->H, p->walk_v, a, p->persistent_blocks, p->walk_lds, s) != hipSuccess)
                return HS_ERR_HIP;
            return from_hip(hsk::launch_plane_counts(out, out_offsets, caps, 0,
                                                     reinterpret_cast<unsigned long long*>(counts), p->n_fops,
                                                     p->H, p->s_bin, (1u << p->s_k) - 1u, s));
        }
        const int64_t* tables = t.batch;
        hipError_t e = hsk::launch_zero_i64(counts, (int64_t)p->n_fops * (p->H + 1), s);
        if (e != hipSuccess) return HS_ERR_HIP;
        hsk::BatchArgs b{};
        b.fops = fops;
        b.lds = lds;
        b.n_chans = tables;
        b.tile_prefix = tables + p->n_fops;
        b.tiles_total = p->tiles_total;
        b.n_fops = p->n_fops;
        b.T = (int32_t)p->T;
        b.c = (int32_t)(p->T / 2);
        b.R = p->tile_rows;
        b.row_blocks = p->row_blocks;
        b.scale = p->scale;
        b.inv_scale = 1.0f / p->scale;
        b.ta = ta;
        b.out = out;
        b.out_offsets = out_offsets;
        b.caps = caps;
        b.counts = reinterpret_cast<unsigned long long*>(counts);
        b.s_row = p->s_row;
        b.s_bin = p->s_bin;
        b.kmask = (1u << p->s_k) - 1u;
        b.table_whole = hsk::table_whole((int)p->T, p->H) ? 1 : 0;
        const int grid = persistent_grid(p, p->tiles_total);
        if (hsk::launch_batched(p->dtype, p->H, b, grid, p->lds_bytes, s) != hipSuccess) return HS_ERR_HIP;
        return from_hip(hsk::launch_plane_counts(out, out_offsets, caps, 0,
                                                 reinterpret_cast<unsigned long long*>(counts), p->n_fops, p->H,
                                                 p->s_bin, b.kmask, s));
    } catch (...) {
        return HS_ERR_HIP;
    }
}

size_t hs_sort_workspace_bytes(int64_t n)
{
    if (n <= 1) return 0;
    size_t bytes = 0;
    if (hsk::sort_workspace(n, &bytes) != hipSuccess) return 0;
    return bytes;
}

hs_status hs_sort_candidates(hs_cand* cand, int64_t n, void* work, void* stream)
{
    if (n < 0 || (n > 1 && (!cand || !work))) return HS_ERR_INVALID;
    try {
        return from_hip(hsk::sort_candidates(reinterpret_cast<uint64_t*>(cand), n, work,
                                             (hipStream_t)stream));
    } catch (...) {
        return HS_ERR_HIP;
    }
}

namespace {
size_t round256(size_t x) { return (x + 255) & ~(size_t)255; }
size_t plane_bytes(const hs_plan* p) { return (size_t)p->T * (size_t)p->N * 4; }
size_t partial_bytes(const hs_plan* p)
{
    return (size_t)hsk::backward_partial_floats((int)p->T, p->H, p->tile_rows, p->N) * 4;
}
bool tau_ok(float tau) { return tau > 0.0f && tau < INFINITY; }
}  // namespace

size_t hs_backward_workspace_bytes(const hs_plan* p)
{
    if (!p || p->n_fops != 0) return 0;
    return round256(partial_bytes(p));
}

hs_status hs_sum_backward(const hs_plan* p, const float* g, float* dfop, void* work, void* stream)
{
    if (!p || p->n_fops != 0 || !g || !dfop) return HS_ERR_INVALID;
    if (p->mapping != HS_MAP_PAPER) return HS_ERR_UNSUPPORTED;
    if (partial_bytes(p) > 0 && !work) return HS_ERR_INVALID;
    try {
        return from_hip(hsk::launch_backward(g, dfop, static_cast<float*>(work), (int)p->T, p->N, p->H,
                                             p->tile_rows, (hipStream_t)stream));
    } catch (...) {
        return HS_ERR_HIP;
    }
}

// Workspace of the statistic: the backward's tile partials (tiles of
// lse_backward_tile_rows() rows) and the fused forward's per-block pairs;
// for 16-bit plans also the H planes the forward materialises, followed by
// the larger of the partials and the plane reduction's pairs.
size_t hs_lse_workspace_bytes(const hs_plan* p)
{
    if (!p || p->n_fops != 0) return 0;
    const size_t bwd = (size_t)hsk::backward_partial_floats((int)p->T, p->H, hsk::lse_backward_tile_rows(), p->N) * 4;
    const size_t fused = (size_t)hsk::kLseMaxBlocks * p->H * 2 * sizeof(float);
    if (p->dtype == HS_DTYPE_F32) return std::max(round256(bwd), round256(fused));
    const size_t tail = std::max(bwd, (size_t)hsk::lse_part_bytes(p->H));
    return round256(plane_bytes(p) * p->H) + round256(tail);
}

namespace {

// Grid of the fused statistic: two blocks per compute unit (the planner's
// LDS budget), at most one per tile and kLseMaxBlocks.
int lse_grid(const hs_plan* p)
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
    int64_t g = p->persistent_blocks > 0 ? p->persistent_blocks : 2 * (int64_t)cus;
    g = std::min<int64_t>(g, std::min<int64_t>(p->tiles_total, hsk::kLseMaxBlocks));
    return (int)std::max<int64_t>(g, 1);
}

// The fused statistic (fp32 plans): the planes are formed tile by tile and
// never stored; `part` holds lse_grid(p) x H (max, sum) pairs.
hs_status lse_forward_fused(const hs_plan* p, const void* fop, int64_t ld, float tau, double* lse, double* loss,
                            float* part, const DevTabs& t, hipStream_t s)
{
    const int g = lse_grid(p);
    hsk::TileArgs a = tile_args(p, fop, ld, t);
    a.lse_part = part;
    a.lse_c = (float)(1.4426950408889634 / (double)p->scale / (double)tau);
    hipError_t e = hsk::launch_fused(hsk::kModeLse, p->dtype, p->H, a, p->tiles_total, g, p->lds_bytes, s);
    if (e != hipSuccess) return HS_ERR_HIP;
    e = hsk::launch_lse_fused_final(a.lse_part, g, p->H, 1.0 / (double)p->scale, (double)tau, lse, s);
    if (e != hipSuccess) return HS_ERR_HIP;
    return loss ? from_hip(hsk::launch_lse_loss(lse, p->H, (double)tau, loss, s)) : HS_OK;
}

}  // namespace

hs_status hs_lse_forward_noalloc(const hs_plan* p, const void* fop, int64_t ld, float tau, double* lse,
                                 double* loss, void* stream)
{
    if (!p || p->n_fops != 0 || !lse || !tau_ok(tau)) return HS_ERR_INVALID;
    if (p->mapping != HS_MAP_PAPER || p->dtype != HS_DTYPE_F32) return HS_ERR_UNSUPPORTED;
    if (!fop_ok(p, fop, ld, p->N)) return HS_ERR_INVALID;
    try {
        hipStream_t s = (hipStream_t)stream;
        if ((size_t)lse_grid(p) * p->H * 2 * sizeof(float) > hsk::kNoAllocScratchBytes) return HS_ERR_INVALID;
        void* scratch = nullptr;
        if (hsk::noalloc_scratch(&scratch) != hipSuccess) return HS_ERR_HIP;
        DevTabs t;
        const hs_status st = device_tables_present(p, s, &t);
        if (st != HS_OK) return st;
        return lse_forward_fused(p, fop, ld, tau, lse, loss, static_cast<float*>(scratch), t, s);
    } catch (...) {
        return HS_ERR_HIP;
    }
}

hs_status hs_lse_forward(const hs_plan* p, const void* fop, int64_t ld, float tau, double* lse,
                         double* loss, void* work, void* stream)
{
    if (!p || p->n_fops != 0 || !lse || !work || !tau_ok(tau)) return HS_ERR_INVALID;
    if (p->mapping != HS_MAP_PAPER) return HS_ERR_UNSUPPORTED;
    if (!fop_ok(p, fop, ld, p->N)) return HS_ERR_INVALID;
    try {
        hipStream_t s = (hipStream_t)stream;
        DevTabs t;
        const hs_status st = device_tables(p, s, &t);
        if (st != HS_OK) return st;
        if (p->dtype == HS_DTYPE_F32) return lse_forward_fused(p, fop, ld, tau, lse, loss, static_cast<float*>(work), t, s);
        float* planes = static_cast<float*>(work);
        void* tail = static_cast<char*>(work) + round256(plane_bytes(p) * p->H);
        hsk::TileArgs a = tile_args(p, fop, ld, t);
        a.hp = planes;
        hipError_t e = hsk::launch_fused(hsk::kModeSum, p->dtype, p->H, a, p->tiles_total,
                                         persistent_grid(p, p->tiles_total), p->lds_bytes, s);
        if (e != hipSuccess) return HS_ERR_HIP;
        e = hsk::launch_lse_reduce(planes, p->T * p->N, p->H, tau, tail, lse, s);
        if (e != hipSuccess) return HS_ERR_HIP;
        return loss ? from_hip(hsk::launch_lse_loss(lse, p->H, (double)tau, loss, s)) : HS_OK;
    } catch (...) {
        return HS_ERR_HIP;
    }
}

hs_status hs_lse_backward(const hs_plan* p, const void* fop, int64_t ld, const double* lse,
                          float tau, const double* gscale, float* dfop, void* work, void* stream)
{
    if (!p || p->n_fops != 0 || !lse || !dfop || !work || !tau_ok(tau)) return HS_ERR_INVALID;
    if (p->mapping != HS_MAP_PAPER) return HS_ERR_UNSUPPORTED;
    if (!fop_ok(p, fop, ld, p->N)) return HS_ERR_INVALID;
    try {
        // the weights are formed inside the transpose's tile pass: no weight
        // plane is written or read back
        return from_hip(hsk::launch_lse_backward_fused(p->dtype, fop, ld, (int)p->T, p->N, p->H, 1.0f / p->scale,
                                                       (double)tau, lse, gscale, dfop, static_cast<float*>(work),
                                                       (hipStream_t)stream));
    } catch (...) {
        return HS_ERR_HIP;
    }
}

hs_status hs_check_counts(const int64_t* counts_host, int32_t n_hp, int64_t capacity)
{
    if (!counts_host || n_hp < 1 || n_hp > hsk::kMaxH || capacity < 0) return HS_ERR_INVALID;
    if (counts_host[n_hp] < 0) return HS_ERR_INVALID;
    return counts_host[n_hp] > capacity ? HS_ERR_OVERFLOW : HS_OK;
}

const char* hs_status_string(hs_status s)
{
    switch (s) {
    case HS_OK: return "ok";
    case HS_ERR_INVALID: return "invalid argument";
    case HS_ERR_OVERFLOW: return "candidate list exceeds capacity";
    case HS_ERR_HIP: return "HIP runtime error";
    case HS_ERR_UNSUPPORTED: return "unsupported";
    case HS_ERR_NOMEM: return "out of memory";
    }
    return "unknown status";
}

hs_status hs_stream_read(const void* src, int64_t bytes, float* sink, int32_t grid, void* stream)
{
    if (!src || !sink || bytes <= 0 || bytes % 16 != 0 || (reinterpret_cast<uintptr_t>(src) & 15) != 0 ||
        grid < 1 || grid > 65536)
        return HS_ERR_INVALID;
    try {
        return from_hip(hsk::launch_stream_read(src, bytes, sink, grid, (hipStream_t)stream));
    } catch (...) {
        return HS_ERR_HIP;
    }
}

const char* hs_version(void) { return "hs-mi355x 0.1.0 (gfx950)"; }

}  // extern "C"
