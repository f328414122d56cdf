// Binning: prefix scans, stable LSD radix sort, key duplication and tile
// ranges (Sec. II-A of the paper: "parallel prefix scan ... duplicates ...
// into key-value pairs, which are sorted by GPU radix sort to produce
// front-to-back index ranges").
//
// Two-stage ordering.  Instead of radix-sorting 64-bit (tile << 32 | depth)
// keys over all P pairs (ceil(log2 tiles) + 32 bits: six 8-bit passes over P),
// the visible Gaussians are first sorted by depth (32-bit key, N elements),
// duplicated in that order, and the pairs are then stably sorted by tile id
// only (ceil(log2 tiles) bits: two passes for 1080p).  Because both sorts
// are stable and duplication follows (depth, id) order, the result is
// identical to the single 64-bit sort.
#include "common.hpp"

namespace lgs {
namespace {

constexpr int kScanItems = 8;                          // per thread
constexpr int kScanTile = kBlock * kScanItems;         // 2048 per block
constexpr int kRadixItems = 16;                        // per thread
constexpr int kRadixTile = kBlock * kRadixItems;       // 4096 per block
constexpr int kRadixBits = 8;
constexpr int kRadixBins = 1 << kRadixBits;

// ---------------------------------------------------------------------------
// block-wide scans (NW wave64 per block)
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v)
{
    const int lane = __lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        T o = __shfl_up(v, off, 64);
        if (lane >= off) v += o;
    }
    return v;
}

template <typename T, int NW>
__device__ __forceinline__ T block_exclusive_scan(T v, T &total, T *s_warp /*[NW]*/)
{
    const int lane = __lane_id(), wid = threadIdx.x >> 6;
    T incl = wave_inclusive_scan(v);
    if (lane == 63) s_warp[wid] = incl;
    __syncthreads();
    T before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        T s = s_warp[w];
        if (w < wid) before += s;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return incl - v + before;
}

__device__ __forceinline__ int64_t live_count(int64_t n_max, const uint32_t *n_dev)
{
    if (!n_dev) return n_max;
    int64_t n = (int64_t)*n_dev;
    return n < n_max ? n : n_max;
}

// ---------------------------------------------------------------------------
// device-wide exclusive scan: reduce -> scan of block partials -> final
// ---------------------------------------------------------------------------
template <typename T, typename L>
__global__ __launch_bounds__(kBlock) void scan_reduce_kernel(L ld, int64_t n_max, const uint32_t *n_dev, T *partials)
{
    __shared__ T s_warp[kBlock / 64];
    const int64_t n = live_count(n_max, n_dev);
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    T sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) sum += ld(base + k);
    T total;
    block_exclusive_scan<T, kBlock / 64>(sum, total, s_warp);
    if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

template <typename T>
__global__ __launch_bounds__(1024) void scan_partials_kernel(T *partials, int64_t nb, T *total_out)
{
    __shared__ T s_warp[16];
    T carry = 0;
    for (int64_t c = 0; c < nb; c += 1024) {
        const int64_t i = c + threadIdx.x;
        T v = i < nb ? partials[i] : (T)0;
        T tot;
        T ex = block_exclusive_scan<T, 16>(v, tot, s_warp);
        if (i < nb) partials[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0 && total_out) *total_out = carry;
}

template <typename T, typename L, typename S>
__global__ __launch_bounds__(kBlock) void scan_final_kernel(L ld, S st, int64_t n_max, const uint32_t *n_dev,
                                                            const T *partials)
{
    __shared__ T s_warp[kBlock / 64];
    const int64_t n = live_count(n_max, n_dev);
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    T item[kScanItems];
    T sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        item[k] = base + k < n ? ld(base + k) : (T)0;
        sum += item[k];
    }
    T total;
    T run = block_exclusive_scan<T, kBlock / 64>(sum, total, s_warp) + partials[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) st(base + k, run, item[k]);
        run += item[k];
    }
}

template <typename T>
struct ArrayLoad {
    const T *p;
    __device__ T operator()(int64_t i) const { return p[i]; }
};
template <typename T>
struct ArrayStore {
    T *p;
    __device__ void operator()(int64_t i, T excl, T) const { p[i] = excl; }
};

// visible <=> non-empty tile rectangle
struct VisibleLoad {
    const int4 *rect;
    __device__ uint32_t operator()(int64_t i) const
    {
        int4 r = rect[i];
        return (r.z > r.x && r.w > r.y) ? 1u : 0u;
    }
};
// compaction of visible Gaussians into (depth bits, id)
struct CompactStore {
    const float *depth;
    uint32_t *keys, *vals;
    __device__ void operator()(int64_t i, uint32_t excl, uint32_t item) const
    {
        if (item) {
            keys[excl] = __float_as_uint(depth[i]);   // depth > znear > 0: bits order like the floats
            vals[excl] = (uint32_t)i;
        }
    }
};
// tiles touched by the r-th Gaussian in depth order
struct PairCountLoad {
    const uint32_t *order;
    const int4 *rect;
    __device__ uint64_t operator()(int64_t r) const
    {
        int4 q = rect[order[r]];
        return (uint64_t)(q.z - q.x) * (uint64_t)(q.w - q.y);
    }
};
// duplication: one (tile, id) pair per touched tile, row-major over the rectangle
struct DuplicateStore {
    const uint32_t *order;
    const int4 *rect;
    int tiles_x;
    uint64_t cap;
    uint32_t *keys, *vals;
    __device__ void operator()(int64_t r, uint64_t excl, uint64_t item) const
    {
        if (!item) return;
        const uint32_t g = order[r];
        const int4 q = rect[g];
        uint64_t o = excl;
        for (int ty = q.y; ty < q.w; ++ty)
            for (int tx = q.x; tx < q.z; ++tx, ++o)
                if (o < cap) {
                    keys[o] = (uint32_t)(ty * tiles_x + tx);
                    vals[o] = g;
                }
    }
};

__global__ void finalize_pairs_kernel(const uint64_t *total, uint64_t cap, int64_t *num_pairs, int32_t *overflow,
                                      uint32_t *n_eff)
{
    const uint64_t p = *total;
    *num_pairs = (int64_t)p;
    *overflow = p > cap ? 1 : 0;
    *n_eff = (uint32_t)(p > cap ? cap : p);
}

// ---------------------------------------------------------------------------
// stable LSD radix sort, 8-bit digits, u32 keys + u32 values
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void radix_hist_kernel(const uint32_t *__restrict__ keys, int64_t n_max,
                                                            const uint32_t *n_dev, int shift,
                                                            uint32_t *__restrict__ hist, int64_t nblocks)
{
    __shared__ uint32_t s_h[kBlock / 64][kRadixBins];
    const int wid = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < (kBlock / 64) * kRadixBins; i += kBlock) (&s_h[0][0])[i] = 0;
    __syncthreads();
    const int64_t n = live_count(n_max, n_dev);
    const int64_t start = (int64_t)blockIdx.x * kRadixTile;
    const int64_t end = start + kRadixTile < n ? start + kRadixTile : n;
    for (int64_t e = start + threadIdx.x; e < end; e += kBlock)
        atomicAdd(&s_h[wid][(keys[e] >> shift) & (kRadixBins - 1)], 1u);
    __syncthreads();
    uint32_t c = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) c += s_h[w][threadIdx.x];
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = c;
}

// Each block re-reads its 4096 elements in 16 rounds of 256 and scatters them
// to digit offset + (elements of that digit before it in the block).  Within a
// round the rank among equal digits comes from eight wave ballots; across
// waves and rounds from per-wave digit counts in LDS.
__global__ __launch_bounds__(kBlock) void radix_scatter_kernel(const uint32_t *__restrict__ keys_in,
                                                               const uint32_t *__restrict__ vals_in,
                                                               uint32_t *__restrict__ keys_out,
                                                               uint32_t *__restrict__ vals_out, int64_t n_max,
                                                               const uint32_t *n_dev, int shift,
                                                               const uint32_t *__restrict__ hist_scan, int64_t nblocks)
{
    __shared__ uint32_t s_base[kRadixBins];
    __shared__ uint32_t s_wc[kBlock / 64][kRadixBins];
    const int64_t n = live_count(n_max, n_dev);
    const int64_t start = (int64_t)blockIdx.x * kRadixTile;
    if (start >= n) return;                                  // uniform across the block
    const int lane = __lane_id(), wid = threadIdx.x >> 6;
    s_base[threadIdx.x] = hist_scan[(int64_t)threadIdx.x * nblocks + blockIdx.x];
    const uint64_t lt = lanemask_lt();
    for (int round = 0; round < kRadixItems; ++round) {
        const int64_t e = start + (int64_t)round * kBlock + threadIdx.x;
        if (start + (int64_t)round * kBlock >= n) break;     // uniform
        const bool active = e < n;
        const uint32_t key = active ? keys_in[e] : 0u;
        const uint32_t val = active ? vals_in[e] : 0u;
        const uint32_t d = (key >> shift) & (kRadixBins - 1);
#pragma unroll
        for (int k = 0; k < kRadixBins / 64; ++k) s_wc[wid][lane + 64 * k] = 0u;
        uint64_t match = __ballot(active);
#pragma unroll
        for (int b = 0; b < kRadixBits; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            match &= bit ? bb : ~bb;
        }
        const uint32_t rank = __popcll(match & lt);
        if (active && rank == 0) s_wc[wid][d] = (uint32_t)__popcll(match);
        __syncthreads();
        if (active) {
            uint32_t before = 0;
#pragma unroll
            for (int w = 0; w < kBlock / 64; ++w) before += (w < wid) ? s_wc[w][d] : 0u;
            const uint32_t pos = s_base[d] + before + rank;
            keys_out[pos] = key;
            vals_out[pos] = val;
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) add += s_wc[w][threadIdx.x];
        s_base[threadIdx.x] += add;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// tile ranges
// ---------------------------------------------------------------------------
__global__ void ranges_kernel(const uint32_t *__restrict__ keys, const int64_t *num_pairs, const int32_t *overflow,
                              int64_t cap, uint2 *__restrict__ ranges)
{
    if (overflow && *overflow) return;
    int64_t n = *num_pairs;
    if (n > cap) n = cap;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t t = keys[i];
        if (i == 0 || keys[i - 1] != t) ranges[t].x = (uint32_t)i;
        if (i == n - 1 || keys[i + 1] != t) ranges[t].y = (uint32_t)(i + 1);
    }
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------
inline size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

struct SortWorkspace {
    uint32_t *dk[2], *dv[2];      // depth keys / ids, ping-pong [n]
    uint32_t *pk, *pv;            // alternate pair buffers [cap]
    uint32_t *hist;               // [256 * nblocks_max]
    uint64_t *partials;           // scan partials
    uint32_t *n_vis;              // visible count
    uint32_t *n_eff;              // min(P, cap)
    uint64_t *p_total;            // P
    size_t bytes;
};

inline int64_t radix_blocks(int64_t n) { return (n + kRadixTile - 1) / kRadixTile; }

SortWorkspace plan_workspace(char *base, int64_t n, int64_t cap)
{
    SortWorkspace w{};
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off += align_up(bytes > 0 ? bytes : 1);
        return p;
    };
    const int64_t nm = n > 0 ? n : 1;
    for (int k = 0; k < 2; ++k) {
        w.dk[k] = (uint32_t *)take(sizeof(uint32_t) * nm);
        w.dv[k] = (uint32_t *)take(sizeof(uint32_t) * nm);
    }
    w.pk = (uint32_t *)take(sizeof(uint32_t) * (cap > 0 ? cap : 1));
    w.pv = (uint32_t *)take(sizeof(uint32_t) * (cap > 0 ? cap : 1));
    const int64_t nbmax = radix_blocks(n > cap ? n : cap) + 1;
    w.hist = (uint32_t *)take(sizeof(uint32_t) * kRadixBins * nbmax);
    int64_t scan_max = kRadixBins * nbmax;
    if (n > scan_max) scan_max = n;
    w.partials = (uint64_t *)take(sizeof(uint64_t) * ((scan_max + kScanTile - 1) / kScanTile + 1));
    w.n_vis = (uint32_t *)take(sizeof(uint32_t));
    w.n_eff = (uint32_t *)take(sizeof(uint32_t));
    w.p_total = (uint64_t *)take(sizeof(uint64_t));
    w.bytes = off;
    return w;
}

// exclusive scan of ld(0..n) with a device-resident count (n_dev may be NULL)
template <typename T, typename L, typename S>
void device_scan(L ld, S st, int64_t n_max, const uint32_t *n_dev, T *partials, T *total, hipStream_t s)
{
    const int64_t nb = (n_max + kScanTile - 1) / kScanTile;
    if (nb == 0) {
        hipLaunchKernelGGL(scan_partials_kernel<T>, dim3(1), dim3(1024), 0, s, partials, (int64_t)0, total);
        return;
    }
    hipLaunchKernelGGL((scan_reduce_kernel<T, L>), dim3((unsigned)nb), dim3(kBlock), 0, s, ld, n_max, n_dev, partials);
    hipLaunchKernelGGL(scan_partials_kernel<T>, dim3(1), dim3(1024), 0, s, partials, nb, total);
    hipLaunchKernelGGL((scan_final_kernel<T, L, S>), dim3((unsigned)nb), dim3(kBlock), 0, s, ld, st, n_max, n_dev,
                       (const T *)partials);
}

// one stable radix pass over [0, min(n_max, *n_dev))
void radix_pass(const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout, int64_t n_max,
                const uint32_t *n_dev, int shift, const SortWorkspace &w, hipStream_t s)
{
    const int64_t nb = radix_blocks(n_max);
    if (nb == 0) return;
    hipLaunchKernelGGL(radix_hist_kernel, dim3((unsigned)nb), dim3(kBlock), 0, s, kin, n_max, n_dev, shift, w.hist, nb);
    device_scan<uint32_t>(ArrayLoad<uint32_t>{w.hist}, ArrayStore<uint32_t>{w.hist}, kRadixBins * nb, nullptr,
                          reinterpret_cast<uint32_t *>(w.partials), (uint32_t *)nullptr, s);
    hipLaunchKernelGGL(radix_scatter_kernel, dim3((unsigned)nb), dim3(kBlock), 0, s, kin, vin, kout, vout, n_max,
                       n_dev, shift, (const uint32_t *)w.hist, nb);
}

}  // namespace
}  // namespace lgs

using namespace lgs;

extern "C" size_t lgs_sort_workspace_size(int64_t n, int64_t capacity_pairs, int32_t num_tiles)
{
    (void)num_tiles;
    if (n < 0 || capacity_pairs < 0) return 0;
    return plan_workspace(nullptr, n, capacity_pairs).bytes;
}

extern "C" lgs_status lgs_sort(int64_t n, int32_t tiles_x, int32_t tiles_y, const float *depth, const int32_t *rect,
                               uint32_t *tile_keys, uint32_t *values, int64_t capacity_pairs, int64_t *num_pairs,
                               int32_t *overflow, void *workspace, size_t workspace_bytes, void *stream)
{
    LGS_REQUIRE(n >= 0 && n < (int64_t)UINT32_MAX, "lgs_sort: n out of range");
    LGS_REQUIRE(tiles_x > 0 && tiles_y > 0 && (int64_t)tiles_x * tiles_y < (1ll << 31), "lgs_sort: bad tile grid");
    LGS_REQUIRE(capacity_pairs >= 0 && capacity_pairs < (int64_t)UINT32_MAX, "lgs_sort: capacity out of range");
    LGS_REQUIRE(num_pairs && overflow, "lgs_sort: null num_pairs/overflow");
    LGS_REQUIRE(n == 0 || (depth && rect), "lgs_sort: null input");
    LGS_REQUIRE(capacity_pairs == 0 || (tile_keys && values), "lgs_sort: null output");
    LGS_REQUIRE(rect == nullptr || (uintptr_t)rect % 16 == 0, "lgs_sort: rect must be 16-byte aligned");
    const size_t need = plan_workspace(nullptr, n, capacity_pairs).bytes;
    LGS_REQUIRE(workspace && workspace_bytes >= need, "lgs_sort: workspace too small (%zu < %zu bytes)",
                workspace_bytes, need);
    LGS_REQUIRE((uintptr_t)workspace % 256 == 0, "lgs_sort: workspace must be 256-byte aligned");
    hipStream_t s = as_stream(stream);
    SortWorkspace w = plan_workspace(static_cast<char *>(workspace), n, capacity_pairs);
    const int4 *rc = reinterpret_cast<const int4 *>(rect);

    // 1. compact visible Gaussians into (depth bits, id)
    device_scan<uint32_t>(VisibleLoad{rc}, CompactStore{depth, w.dk[0], w.dv[0]}, n, nullptr,
                          reinterpret_cast<uint32_t *>(w.partials), w.n_vis, s);
    // 2. stable sort by depth: four 8-bit passes, result back in buffer 0
    for (int pass = 0; pass < 4; ++pass) {
        const int a = pass & 1;
        radix_pass(w.dk[a], w.dv[a], w.dk[a ^ 1], w.dv[a ^ 1], n, w.n_vis, 8 * pass, w, s);
    }
    // 3. scan of tile counts in depth order, fused with duplication.  The
    //    number of tile-sort passes decides which buffer receives the pairs so
    //    that the sorted result ends in the caller's buffers.
    int bits = 1;
    while ((1ll << bits) < (int64_t)tiles_x * tiles_y) ++bits;
    const int passes = (bits + kRadixBits - 1) / kRadixBits;
    uint32_t *k0 = (passes & 1) ? w.pk : tile_keys, *v0 = (passes & 1) ? w.pv : values;
    uint32_t *k1 = (passes & 1) ? tile_keys : w.pk, *v1 = (passes & 1) ? values : w.pv;
    device_scan<uint64_t>(PairCountLoad{w.dv[0], rc}, DuplicateStore{w.dv[0], rc, tiles_x, (uint64_t)capacity_pairs, k0, v0},
                          n, w.n_vis, w.partials, w.p_total, s);
    hipLaunchKernelGGL(finalize_pairs_kernel, dim3(1), dim3(1), 0, s, (const uint64_t *)w.p_total,
                       (uint64_t)capacity_pairs, num_pairs, overflow, w.n_eff);
    // 4. stable sort of the pairs by tile id
    for (int pass = 0; pass < passes; ++pass) {
        if (pass & 1) radix_pass(k1, v1, k0, v0, capacity_pairs, w.n_eff, 8 * pass, w, s);
        else radix_pass(k0, v0, k1, v1, capacity_pairs, w.n_eff, 8 * pass, w, s);
    }
    LGS_LAUNCHED("lgs_sort");
    return LGS_OK;
}

extern "C" lgs_status lgs_tile_ranges(const uint32_t *tile_keys, const int64_t *num_pairs, const int32_t *overflow,
                                      int64_t capacity_pairs, int32_t num_tiles, uint32_t *ranges, void *stream)
{
    LGS_REQUIRE(num_tiles > 0 && ranges && num_pairs, "lgs_tile_ranges: bad arguments");
    LGS_REQUIRE(capacity_pairs >= 0 && (capacity_pairs == 0 || tile_keys), "lgs_tile_ranges: bad pair buffer");
    LGS_REQUIRE((uintptr_t)ranges % 8 == 0, "lgs_tile_ranges: ranges must be 8-byte aligned");
    hipStream_t s = as_stream(stream);
    fill_async<uint64_t>(reinterpret_cast<uint64_t *>(ranges), 0ull, num_tiles, s);
    if (capacity_pairs > 0) {
        unsigned g = grid_for(capacity_pairs, 256);
        if (g > 8192) g = 8192;
        hipLaunchKernelGGL(ranges_kernel, dim3(g), dim3(256), 0, s, tile_keys, num_pairs, overflow, capacity_pairs,
                           reinterpret_cast<uint2 *>(ranges));
    }
    LGS_LAUNCHED("lgs_tile_ranges");
    return LGS_OK;
}
