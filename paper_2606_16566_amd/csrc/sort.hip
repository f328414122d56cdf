// Binning: prefix scans, stable LSD radix sort, key duplication and tile
// ranges (Sec. II-A of the paper: a parallel prefix scan drives the
// duplication of every Gaussian into key/value pairs, one per touched tile,
// which a GPU radix sort orders front to back within each tile; tile ranges
// are then read off the sorted keys).
//
// Two-stage ordering.  Instead of radix-sorting 64-bit (tile << 32 | depth)
// keys over all P pairs (ceil(log2 tiles) + 32 bits: six 8-bit passes over P),
// the Gaussians are first sorted by depth (32-bit key over N; culled ones
// carry depth +inf and sink to the end) and the pairs, emitted in that order,
// are then ordered stably by tile only.  For grids up to 256 tiles wide the
// pairs are generated straight into tile-column order (the column pass) and
// one stable radix pass on the tile row follows (one pass at 1080p); wider
// grids store the duplicated pairs and sort them by tile id.  Every step is
// stable and the emission follows (depth, id) order, so the result is
// identical to the single 64-bit sort.  The depth sort also brings the tile
// rectangles into depth order, packed into 32 bits and carried as a third
// payload of its passes when every view is at most 256 tiles wide and high
// (coalesced, where a gather by the sorted ids would read a whole cache line
// per 16-byte rectangle), otherwise gathered by its last pass.
#include <mutex>
#include <type_traits>

#include "common.hpp"
#include "render_common.hpp"

namespace lgs {
namespace {

constexpr int kScanItems = 8;                          // per thread
constexpr int kScanTile = kBlock * kScanItems;         // 2048 per block
// Radix blocks (one histogram partition each) hold 256 * ITEMS elements, in
// two tiers by input length: 2048 below 2^22 elements, so that enough blocks
// exist to fill the chip; 8192 beyond, which cuts the per-block histogram
// traffic and lengthens the digit runs that the scatter writes contiguously.
// The scatters use 1024-thread workgroups (2 and 8 elements per thread): more
// waves per block than the histogram's 256 threads, with registers and LDS
// low enough for two resident blocks per CU.  Each tier was the fastest
// measured at its size (a middle tier of 4096 on 512 threads was slower from
// 2^22 up).
constexpr int kRadixItems = 8;                         // smallest tier
constexpr int kRadixTile = kBlock * kRadixItems;       // 2048 per block
constexpr int64_t kLargeRadixFrom = 1 << 22;           // elements
constexpr int kRadixBits = 8;
constexpr int kRadixBins = 1 << kRadixBits;
constexpr int kWaves = kBlock / 64;

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

// v + (v of the lane the DPP control selects), 0 where it selects none or the
// row is masked off (all 64 lanes must be active)
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_add(uint32_t v)
{
    return v + (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xF, false);
}

// 32-bit inclusive scan over the wavefront in DPP steps: shifts by 1, 2, 4, 8
// within each row of 16, then the last lane of rows 0 and 2 into rows 1 and 3
// (row_bcast:15) and lane 31 into rows 2 and 3 (row_bcast:31)
template <>
__device__ __forceinline__ uint32_t wave_inclusive_scan<uint32_t>(uint32_t v)
{
    v = dpp_add<0x111, 0xF>(v);   // row_shr:1
    v = dpp_add<0x112, 0xF>(v);   // row_shr:2
    v = dpp_add<0x114, 0xF>(v);   // row_shr:4
    v = dpp_add<0x118, 0xF>(v);   // row_shr:8
    v = dpp_add<0x142, 0xA>(v);   // row_bcast:15
    v = dpp_add<0x143, 0xC>(v);   // row_bcast:31
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

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// device-wide exclusive scan: reduce -> scan of block partials -> final
// ---------------------------------------------------------------------------
template <typename T, typename L>
__global__ __launch_bounds__(kBlock) void scan_reduce_kernel(L ld, int64_t n_max, const uint32_t *n_dev, T *partials)
{
    __shared__ T s_warp[kWaves];
    const int64_t n = live_count(n_max, n_dev);
    // only the block total is needed here, so lanes read consecutive
    // elements (coalesced) rather than the per-thread runs of the final pass
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x;
    T sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k * kBlock < n) sum += ld(base + k * kBlock);
    T total;
    block_exclusive_scan<T, kWaves>(sum, total, s_warp);
    if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

template <typename T, typename L, typename S>
__global__ __launch_bounds__(kBlock) void scan_final_kernel(L ld, S st, int64_t n_max, const uint32_t *n_dev,
                                                            const T *partials)
{
    __shared__ T s_warp[kWaves];
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
    T run = block_exclusive_scan<T, kWaves>(sum, total, s_warp) + partials[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) st(base + k, run, item[k]);
        run += item[k];
    }
}

// tiles touched by the r-th Gaussian in depth order; the reduce pass gathers
// the rectangle and leaves the count in `cnt` for the final pass
struct PairCountGather {
    const int4 *rect;           // rectangles in depth order
    uint32_t *cnt;
    __device__ uint64_t operator()(int64_t r) const
    {
        const int4 q = rect[r];
        const uint32_t c = (q.z > q.x && q.w > q.y) ? (uint32_t)((q.z - q.x) * (q.w - q.y)) : 0u;
        cnt[r] = c;
        return c;
    }
};
struct U32Load {
    const uint32_t *p;
    __device__ uint64_t operator()(int64_t i) const { return p[i]; }
};
// exclusive pair offsets (in place over the counts), saturated at the capacity
struct OffsetStore {
    uint32_t *off;
    uint64_t cap;
    __device__ void operator()(int64_t r, uint64_t excl, uint64_t) const
    {
        off[r] = (uint32_t)(excl < cap ? excl : cap);
    }
};

// scan of the block partials of the pair counts, which also publishes the
// pair total, the overflow flag and min(P, capacity)
__global__ __launch_bounds__(1024) void pair_partials_kernel(uint64_t *partials, int64_t nb, uint64_t *total_out,
                                                             uint64_t cap, int64_t *num_pairs, int32_t *overflow,
                                                             uint32_t *n_eff)
{
    __shared__ uint64_t s_warp[16];
    uint64_t carry = 0;
    for (int64_t c = 0; c < nb; c += 1024) {
        const int64_t i = c + threadIdx.x;
        const uint64_t v = i < nb ? partials[i] : 0ull;
        uint64_t tot;
        const uint64_t ex = block_exclusive_scan<uint64_t, 16>(v, tot, s_warp);
        if (i < nb) partials[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        *total_out = carry;
        *num_pairs = (int64_t)carry;
        *overflow = carry > cap ? 1 : 0;
        *n_eff = (uint32_t)(carry > cap ? cap : carry);
    }
}

// ---------------------------------------------------------------------------
// Duplication: one (tile, id) pair per touched tile, row-major over the
// Gaussian's tile rectangle, Gaussians in depth order.  Each block owns 256
// consecutive Gaussians and their pair range; every lane emits 4 consecutive
// pairs, locating the first one's Gaussian by binary search over the block's
// offsets in LDS and stepping through the rectangle from there, so stores
// are coalesced and a splat covering many tiles is spread over the block.
// ---------------------------------------------------------------------------
constexpr int kDupPerLane = 4;

// Tile grids of a view batch: element e = v * per_view + g belongs to view v,
// whose tiles are the global ids [tile_off[v], tile_off[v] + tx * ty).
struct TileGrids {
    uint32_t per_view;
    int V;
    int tile_off[kMaxViews];
    int tiles_x[kMaxViews];
    int row_off[kMaxViews];     // first global tile row of each view (rows of all views stacked)
};

__global__ __launch_bounds__(kBlock) void duplicate_kernel(const uint32_t *__restrict__ order,
                                                           const int4 *__restrict__ rect,
                                                           const uint32_t *__restrict__ off,
                                                           const uint64_t *p_total, uint64_t cap, TileGrids tg,
                                                           int64_t n, uint32_t *__restrict__ keys,
                                                           uint32_t *__restrict__ vals)
{
    __shared__ uint32_t s_off[kBlock + 1];
    __shared__ int4 s_rect[kBlock];
    __shared__ uint32_t s_id[kBlock];
    __shared__ int2 s_grid[kBlock];     // (first global tile, tiles_x) of the element's view
    const int64_t first = (int64_t)blockIdx.x * kBlock;
    if (first >= n) return;
    const int cnt = (int)min((int64_t)kBlock, n - first);
    const uint64_t total = *p_total;
    const uint32_t lim = (uint32_t)(total < cap ? total : cap);
    if ((int)threadIdx.x < cnt) {
        const uint32_t g = order[first + threadIdx.x];
        const int v = tg.V > 1 ? (int)(g / tg.per_view) : 0;
        s_id[threadIdx.x] = g;
        s_rect[threadIdx.x] = rect[first + threadIdx.x];
        s_grid[threadIdx.x] = make_int2(tg.tile_off[v], tg.tiles_x[v]);
        s_off[threadIdx.x] = off[first + threadIdx.x];
    }
    if (threadIdx.x == 0) s_off[cnt] = first + cnt < n ? off[first + cnt] : lim;
    __syncthreads();
    const uint32_t beg = s_off[0], end = s_off[cnt];
    // lanes take aligned groups of 4 positions so interior groups are written
    // with 16-byte stores
    const uint32_t g0 = beg / kDupPerLane, g1 = (end + kDupPerLane - 1) / kDupPerLane;
    for (uint32_t grp = g0 + threadIdx.x; grp < g1; grp += kBlock) {
        const uint32_t pa = grp * kDupPerLane;
        const uint32_t p0 = pa > beg ? pa : beg;          // first position of this group in range
        if (p0 >= end) continue;
        // last Gaussian k with s_off[k] <= p0 (a Gaussian without pairs shares
        // its successor's offset, so the last of a run of equal offsets owns p0)
        int lo = 0, hi = cnt - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_off[mid] <= p0) lo = mid; else hi = mid - 1;
        }
        int k = lo;
        int4 q = s_rect[k];
        uint32_t w = (uint32_t)(q.z - q.x);
        const uint32_t i = p0 - s_off[k];
        uint32_t ty = i / w, tx = i - ty * w;
        uint32_t kk[kDupPerLane], vv[kDupPerLane];
#pragma unroll
        for (int e = 0; e < kDupPerLane; ++e) {
            const uint32_t p = pa + e;
            kk[e] = 0u; vv[e] = 0u;
            if (p < p0 || p >= end) continue;
            while (p >= s_off[k + 1]) {                 // next Gaussian that has pairs
                ++k;
                q = s_rect[k];
                w = (uint32_t)(q.z - q.x);
                tx = 0; ty = 0;
            }
            const int2 gr = s_grid[k];
            kk[e] = (uint32_t)(gr.x + (q.y + (int)ty) * gr.y + q.x + (int)tx);
            vv[e] = s_id[k];
            if (++tx == w) { tx = 0; ++ty; }
        }
        if (pa >= beg && pa + kDupPerLane <= end) {
            *reinterpret_cast<uint4 *>(keys + pa) = make_uint4(kk[0], kk[1], kk[2], kk[3]);
            *reinterpret_cast<uint4 *>(vals + pa) = make_uint4(vv[0], vv[1], vv[2], vv[3]);
        } else {
#pragma unroll
            for (int e = 0; e < kDupPerLane; ++e) {
                const uint32_t p = pa + e;
                if (p >= p0 && p < end) { keys[p] = kk[e]; vals[p] = vv[e]; }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort, 8-bit digits, u32 keys + u32 values.
// One pass = histogram (per block, digit-major [256][nblocks]) -> per-digit
// row scan (one workgroup per digit, also writes the digit totals) ->
// scatter (each block derives its digit bases from the totals).
// ---------------------------------------------------------------------------

// active lanes of this round of 64 whose digit (nbits <= 8 bits) equals this
// lane's: one ballot per digit bit (unrolled), each keeping the lanes whose
// bit agrees with this lane's: match &= ~(ballot ^ (bit ? ~0 : 0))
__device__ __forceinline__ uint64_t digit_match(bool active, uint32_t d, int nbits)
{
    uint64_t match = __ballot(active);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
        if (b >= nbits) break;
        const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe((int)d, b, 1);   // all ones iff the bit is set
        const uint64_t bb = __ballot(m != 0u);
        match &= ~(bb ^ (((uint64_t)m << 32) | m));
    }
    return match;
}

// Digit plan of the depth passes.  Only the bits in which the visible depth
// keys differ need sorting: with lo and hi the smallest and largest key below
// +inf's bit pattern (positive finite depths order like their bits), the
// first pass rebases every key to key - lo, and every other key (culled:
// +inf) to hi - lo, the largest rebased value (culled Gaussians have no tiles,
// so where they end up among the largest keys changes no pair list); the four
// passes split the bit length of hi - lo as evenly as they can (25 bits: 6,
// 6, 6, 7), so that each pass has fewer distinct digits and longer digit runs
// to write than a fixed 8 bits.  range == nullptr: keys as they are, the
// caller's shift and width.
constexpr uint32_t kInfBits = 0x7F800000u;
struct DepthPlan {
    const uint32_t *range;     // [lo, hi, visible count] (device), from the range kernels
    int pass;                  // 0..3; pass 0 rebases the keys it reads
    bool drop;                 // pass 0 leaves the culled keys out (the later passes take the visible count)
};
struct DigitSel {
    int shift, nbits;
    uint32_t mask, lo, top;    // top = hi - lo: the rebased value of culled keys
    bool rebase, drop;
    __device__ __forceinline__ uint32_t key(uint32_t k) const { return rebase ? (k < kInfBits ? k - lo : top) : k; }
    __device__ __forceinline__ uint32_t digit(uint32_t k) const { return (key(k) >> shift) & mask; }
    __device__ __forceinline__ bool keep(uint32_t k) const { return !drop || k < kInfBits; }   // k: as read
};
template <bool PLAN>
__device__ __forceinline__ DigitSel digit_sel(const DepthPlan &dp, int shift, int nbits)
{
    DigitSel d{shift, nbits, nbits >= 32 ? ~0u : (1u << nbits) - 1u, 0u, 0u, false, false};
    if constexpr (!PLAN) return d;
    const uint32_t lo = dp.range[0], hi = dp.range[1];
    const uint32_t span = hi >= lo ? hi - lo : 0u;         // no visible key: all rebase to 0
    const int bits = span ? 32 - __builtin_clz(span) : 0;
    // the remainder bits go to the last passes, whose digits (exponent and
    // leading mantissa bits) take fewer distinct values than the low ones
    auto width = [&](int p) { return bits / 4 + (p >= 4 - bits % 4 ? 1 : 0); };
    int sh = 0;
    for (int p = 0; p < dp.pass; ++p) sh += width(p);
    d.shift = sh;
    d.nbits = width(dp.pass);
    d.mask = (1u << d.nbits) - 1u;
    d.lo = hi >= lo ? lo : 0u;
    d.top = span;
    d.rebase = dp.pass == 0;
    d.drop = dp.drop && dp.pass == 0;
    // uniform across the wavefront (scalar registers: the digit loops stay
    // uniform branches)
    d.shift = __builtin_amdgcn_readfirstlane(d.shift);
    d.nbits = __builtin_amdgcn_readfirstlane(d.nbits);
    d.mask = (uint32_t)__builtin_amdgcn_readfirstlane((int)d.mask);
    d.lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)d.lo);
    d.top = (uint32_t)__builtin_amdgcn_readfirstlane((int)d.top);
    return d;
}

// [lo, hi] of the keys below +inf's bit pattern, in two steps without
// atomics (thousands of atomics on one address would serialise): per
// workgroup over a grid-stride loop (16-byte loads where aligned) into
// parts[workgroup], then one workgroup over the parts.
constexpr int kRangeParts = 1024;                          // workgroups of the first step, at most
constexpr int64_t kPlanFrom = 1 << 20;                     // Gaussians from which the depth passes take the plan

__device__ __forceinline__ void range_reduce(uint32_t &lo, uint32_t &hi, uint32_t &cnt, uint4 *s_part)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lo = min(lo, (uint32_t)__shfl_xor((int)lo, off, 64));
        hi = max(hi, (uint32_t)__shfl_xor((int)hi, off, 64));
        cnt += (uint32_t)__shfl_xor((int)cnt, off, 64);
    }
    const int wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (__lane_id() == 0) s_part[wid] = make_uint4(lo, hi, cnt, 0u);
    __syncthreads();
    lo = 0xFFFFFFFFu;
    hi = 0u;
    cnt = 0u;
    for (int w = 0; w < nw; ++w) {
        lo = min(lo, s_part[w].x);
        hi = max(hi, s_part[w].y);
        cnt += s_part[w].z;
    }
}

__global__ __launch_bounds__(kBlock) void depth_range_kernel(const uint32_t *__restrict__ keys, int64_t n,
                                                             uint4 *__restrict__ parts)
{
    __shared__ uint4 s_part[kBlock / 64];
    uint32_t lo = 0xFFFFFFFFu, hi = 0u, cnt = 0u;
    auto take = [&](uint32_t k) {
        if (k < kInfBits) { lo = min(lo, k); hi = max(hi, k); ++cnt; }
    };
    const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x, nth = (int64_t)gridDim.x * kBlock;
    int64_t head = 0;
    if (reinterpret_cast<uintptr_t>(keys) % 16 == 0) {
        const uint4 *k4 = reinterpret_cast<const uint4 *>(keys);
        const int64_t n4 = n / 4;
        int64_t i = tid;
        for (; i + 3 * nth < n4; i += 4 * nth) {             // four loads in flight
            uint4 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = k4[i + u * nth];
#pragma unroll
            for (int u = 0; u < 4; ++u) { take(v[u].x); take(v[u].y); take(v[u].z); take(v[u].w); }
        }
        for (; i < n4; i += nth) {
            const uint4 v = k4[i];
            take(v.x); take(v.y); take(v.z); take(v.w);
        }
        head = n4 * 4;
    }
    for (int64_t i = head + tid; i < n; i += nth) take(keys[i]);
    range_reduce(lo, hi, cnt, s_part);
    if (threadIdx.x == 0) parts[blockIdx.x] = make_uint4(lo, hi, cnt, 0u);
}

// range = [lo, hi, visible count] over parts[0, nparts); lo, hi =
// (0xFFFFFFFF, 0) when there is no visible key (or no part)
__global__ __launch_bounds__(kRangeParts) void depth_range_final_kernel(const uint4 *__restrict__ parts,
                                                                        int nparts, uint32_t *__restrict__ range)
{
    __shared__ uint4 s_part[kRangeParts / 64];
    uint32_t lo = 0xFFFFFFFFu, hi = 0u, cnt = 0u;
    if ((int)threadIdx.x < nparts) {
        const uint4 p = parts[threadIdx.x];
        lo = p.x;
        hi = p.y;
        cnt = p.z;
    }
    range_reduce(lo, hi, cnt, s_part);
    if (threadIdx.x == 0) {
        range[0] = lo;
        range[1] = hi;
        range[2] = cnt;
    }
}

// Four consecutive keys of type KT (uint32_t or uint16_t) in one vector load.
template <typename KT> struct Key4;
template <> struct Key4<uint32_t> {
    using V = uint4;
    __device__ static uint32_t at(const V &v, int e) { return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w; }
};
template <> struct Key4<uint16_t> {
    using V = uint2;
    __device__ static uint32_t at(const V &v, int e)
    {
        const uint32_t w = (e < 2) ? v.x : v.y;
        return (e & 1) ? (w >> 16) : (w & 0xFFFFu);
    }
};

// Per-block digit histograms (per-wavefront sub-histograms in LDS, so the
// atomics of one wavefront never contend with another's, optionally split
// further into bank-staggered copies).  One workgroup counts HG consecutive
// blocks: with HG = kHistGroup it writes their counts of each digit as one
// 16-byte row segment, hist[digit * stride + block], stride a multiple of
// kHistGroup (single 4-byte writes at a stride of a whole row would each cost
// a partial cache-line write); short inputs use HG = 1 for more workgroups.
constexpr int kHistGroup = 4;

inline int64_t hist_stride(int64_t nblocks) { return (nblocks + kHistGroup - 1) / kHistGroup * kHistGroup; }

template <int ITEMS, typename KT, int COPIES, int HG, bool PLAN>
__global__ __launch_bounds__(kBlock) void radix_hist_kernel(const KT *__restrict__ keys, int64_t n_max,
                                                            const uint32_t *n_dev, int shift, int nbits,
                                                            uint32_t *__restrict__ hist, int64_t stride,
                                                            DepthPlan dp)
{
    const DigitSel ds = digit_sel<PLAN>(dp, shift, nbits);
    using V = typename Key4<KT>::V;
    constexpr int kTileN = kBlock * ITEMS;
    constexpr int kV = ITEMS / 4;                              // 4-key loads per thread and block
    // COPIES counters per digit and wavefront, lane l counting into copy
    // l % COPIES; the copies are kCopyStride words apart (odd), so the lanes
    // of one digit hit different banks: keys with few distinct digits (the
    // top digit of a key) would otherwise serialise the LDS atomics
    constexpr int kHistCopies = COPIES;
    constexpr int kCopyStride = kRadixBins + (COPIES > 1 ? 1 : 0);
    constexpr int kSubHists = kWaves * kHistCopies;
    __shared__ uint32_t s_h[kSubHists * kCopyStride];
    const int wid = threadIdx.x >> 6, lane = __lane_id();
    uint32_t *my_h = s_h + (wid * kHistCopies + (lane & (kHistCopies - 1))) * kCopyStride;
    const int64_t n = live_count(n_max, n_dev);
    const int64_t g0 = (int64_t)blockIdx.x * HG * kTileN;
    auto aligned = [&](int64_t start) { return (reinterpret_cast<uintptr_t>(keys + start) % sizeof(V)) == 0; };
    // the keys of block j + 1 are in flight while block j is counted
    auto load = [&](int j, V *v) {
        const int64_t start = g0 + (int64_t)j * kTileN;
        const V *k4 = reinterpret_cast<const V *>(keys + start);
        const bool full = start + kTileN <= n && aligned(start);
#pragma unroll
        for (int r = 0; r < kV; ++r) v[r] = full ? k4[r * kBlock + threadIdx.x] : V{};
    };
    V cur[kV], nxt[kV];
    load(0, cur);
    uint32_t c[HG];
#pragma unroll
    for (int j = 0; j < HG; ++j) {
        if (j + 1 < HG) load(j + 1, nxt);
        for (int k = threadIdx.x; k < kSubHists * kCopyStride; k += kBlock) s_h[k] = 0u;
        __syncthreads();
        const int64_t start = g0 + (int64_t)j * kTileN;
        if (start < n) {
            const int cnt = (int)min((int64_t)kTileN, n - start);
            if (cnt == kTileN && aligned(start)) {
#pragma unroll
                for (int r = 0; r < kV; ++r) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const uint32_t k = Key4<KT>::at(cur[r], e);
                        if (!PLAN || ds.keep(k)) atomicAdd(&my_h[ds.digit(k)], 1u);
                    }
                }
            } else {
                const KT *kp = keys + start;
                for (int e = threadIdx.x; e < cnt; e += kBlock) {
                    const uint32_t k = (uint32_t)kp[e];
                    if (!PLAN || ds.keep(k)) atomicAdd(&my_h[ds.digit(k)], 1u);
                }
            }
        }
        __syncthreads();
        c[j] = 0u;
#pragma unroll
        for (int h = 0; h < kSubHists; ++h) c[j] += s_h[h * kCopyStride + threadIdx.x];
        __syncthreads();                                       // before the next block re-zeroes
#pragma unroll
        for (int r = 0; r < kV; ++r) cur[r] = nxt[r];
    }
    if constexpr (HG == kHistGroup)
        *reinterpret_cast<uint4 *>(hist + (int64_t)threadIdx.x * stride + (int64_t)blockIdx.x * kHistGroup) =
            make_uint4(c[0], c[1], c[2], c[3]);
    else
        hist[(int64_t)threadIdx.x * stride + blockIdx.x] = c[0];
}

// Exclusive scan, in place, of one row of per-block counts over the blocks
// that hold elements, in chunks of kBlock * KP: wavefront w takes the chunk's
// w-th quarter, lane-contiguous (coalesced) in KP rounds of 64, scans each
// round across its lanes with a running carry, and the wavefront totals are
// combined through LDS.  The next chunk's counts are loaded while this one
// is scanned.
template <int KP>
__device__ __forceinline__ void radix_rowscan_body(uint32_t *__restrict__ hist, int64_t stride, int64_t n_max,
                                                   const uint32_t *n_dev, int tile_n,
                                                   uint32_t *__restrict__ digit_total)
{
    constexpr int64_t kChunk = (int64_t)kBlock * KP;
    __shared__ uint32_t s_warp[kWaves];
    const int lane = __lane_id(), wid = threadIdx.x >> 6;
    uint32_t *row = hist + (int64_t)blockIdx.x * stride;
    const int64_t n = live_count(n_max, n_dev);
    const int64_t live = (n + tile_n - 1) / tile_n;
    auto at = [&](int64_t c, int k) { return c + (int64_t)wid * 64 * KP + (int64_t)k * 64 + lane; };
    auto load = [&](int64_t c, uint32_t *d) {
#pragma unroll
        for (int k = 0; k < KP; ++k) d[k] = at(c, k) < live ? row[at(c, k)] : 0u;
    };
    uint32_t v[KP], nx[KP];
    load(0, v);
    uint32_t carry = 0;
    for (int64_t c = 0; c < live; c += kChunk) {
        if (c + kChunk < live) load(c + kChunk, nx);
        uint32_t wrun = 0;                                   // this wavefront's running sum
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            const uint32_t incl = wave_inclusive_scan(v[k]);
            const uint32_t x = v[k];
            v[k] = wrun + incl - x;                          // exclusive within the wavefront's quarter
            wrun += (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
        }
        if (lane == 0) s_warp[wid] = wrun;
        __syncthreads();
        uint32_t before = carry, tot = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            const uint32_t t = s_warp[w];
            if (w < wid) before += t;
            tot += t;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KP; ++k)
            if (at(c, k) < live) row[at(c, k)] = before + v[k];
        carry += tot;
#pragma unroll
        for (int k = 0; k < KP; ++k) v[k] = nx[k];
    }
    if (threadIdx.x == 0) digit_total[blockIdx.x] = carry;
}

__global__ __launch_bounds__(kBlock) void radix_rowscan_kernel(uint32_t *__restrict__ hist, int64_t stride,
                                                               int64_t n_max, const uint32_t *n_dev, int tile_n,
                                                               uint32_t *__restrict__ digit_total)
{
    radix_rowscan_body<8>(hist, stride, n_max, n_dev, tile_n, digit_total);
}

// Tile rectangles packed in 32 bits for views at most 256 tiles wide and
// high: first column | (width - 1) << 8 | first row << 16 | (height - 1) << 24,
// kEmptyRect when the rectangle is empty (no valid rectangle packs to it: a
// first column of 255 implies a width of 1).  Columns are clamped to
// [0, 256] and rows to [0, 256) with at most 256 of them, no-ops for
// projected rectangles of such views.
constexpr uint32_t kEmptyRect = 0xFFFFFFFFu;

__device__ __forceinline__ uint32_t pack_rect(int4 q)
{
    q.x = min(max(q.x, 0), 256);
    q.z = min(max(q.z, q.x), 256);
    if (!(q.z > q.x && q.w > q.y)) return kEmptyRect;
    const int y0 = min(max(q.y, 0), 255);
    const int y1 = min(max(q.w, y0 + 1), y0 + 256);
    return (uint32_t)q.x | ((uint32_t)(q.z - q.x - 1) << 8) | ((uint32_t)y0 << 16) | ((uint32_t)(y1 - y0 - 1) << 24);
}

__device__ __forceinline__ int4 unpack_rect(uint32_t p)
{
    if (p == kEmptyRect) return make_int4(0, 0, 0, 0);
    const int x0 = (int)(p & 255u), y0 = (int)((p >> 16) & 255u);
    return make_int4(x0, y0, x0 + (int)((p >> 8) & 255u) + 1, y0 + (int)(p >> 24) + 1);
}

// Optional third payload of a scatter pass (32 bits per element): read from
// in, or, in the first pass, packed from the rectangle of the element's index
// (pack); written to out in sorted order.  out == nullptr: none.
struct AuxPayload {
    const uint32_t *in = nullptr;
    uint32_t *out = nullptr;
    const int4 *pack = nullptr;
};

// Stable scatter of one block of 256 * ITEMS elements.  Wavefront w owns a
// contiguous quarter of the block and ranks its keys in rounds of 64 against
// its own running digit counts, so no workgroup barrier is needed while
// ranking.  The block then orders its elements by digit in LDS (a local
// counting sort) and writes each digit run to its global offset with
// consecutive lanes on consecutive addresses: first the keys, then the
// values through the same LDS buffer, which halves the LDS footprint and
// leaves room for more resident workgroups.  vals_in == nullptr means the
// values are the element indices.  With gather_dst set, the 16-byte record
// gather_src[value] of every element is also written to its sorted place.
// Keys of the column-first binning (below) are (global tile row << 8) |
// tile column; the last pass over them writes tile ids instead.  For view v,
// whose rows start at global row row_off[v], the tile id of global row g and
// column c is base[v] + g * tiles_x[v] + c with base[v] = tile_off[v] -
// row_off[v] * tiles_x[v].  V == 0: keys pass through unchanged (the
// scatter without the mapping is a separate instantiation).
struct RowMap {
    int V;
    int row_off[kMaxViews];
    int base[kMaxViews];
    int tiles_x[kMaxViews];
    // copy of the tables in LDS (s[0..3 * kMaxViews)), by one thread
    __device__ __forceinline__ void stage(int *s) const
    {
#pragma unroll
        for (int v = 0; v < kMaxViews; ++v) {
            s[v] = row_off[v];
            s[kMaxViews + v] = base[v];
            s[2 * kMaxViews + v] = tiles_x[v];
        }
    }
    // tile id of a key; the view by binary search over the staged row offsets
    __device__ __forceinline__ uint32_t tile_of(uint32_t key, const int *s) const
    {
        const uint32_t g = key >> 8, c = key & 255u;
        if (V == 1) return g * (uint32_t)tiles_x[0] + c;
        int v = 0;
#pragma unroll
        for (int step = kMaxViews / 2; step > 0; step >>= 1)
            if (v + step < V && (int)g >= s[v + step]) v += step;
        return (uint32_t)s[kMaxViews + v] + g * (uint32_t)s[2 * kMaxViews + v] + c;
    }
};

template <int ITEMS, int NT, bool MAP, typename KT, bool PLAN>
__global__ __launch_bounds__(NT) void radix_scatter_kernel(const KT *__restrict__ keys_in,
                                                           const uint32_t *__restrict__ vals_in,
                                                           uint32_t *__restrict__ keys_out,
                                                           uint32_t *__restrict__ vals_out, int64_t n_max,
                                                           const uint32_t *n_dev, int shift, int nbits,
                                                           const uint32_t *__restrict__ hist_scan,
                                                           const uint32_t *__restrict__ digit_total,
                                                           int64_t stride, const int4 *__restrict__ gather_src,
                                                           int4 *__restrict__ gather_dst, RowMap rows,
                                                           AuxPayload aux, DepthPlan dp)
{
    constexpr int kW = NT / 64;                             // wavefronts per workgroup
    constexpr int kTileN = NT * ITEMS;
    constexpr int kPerWave = kTileN / kW;
    const DigitSel ds = digit_sel<PLAN>(dp, shift, nbits);
    __shared__ uint32_t s_wc[kW][kRadixBins];              // running, then exclusive-over-waves counts
    __shared__ uint32_t s_lbase[kRadixBins];               // block-local digit offsets
    __shared__ uint32_t s_gbase[kRadixBins];               // global digit offsets of this block
    __shared__ uint32_t s_buf[kTileN];                     // keys, then values, in digit order
    __shared__ uint8_t s_dig[kTileN];                      // digit of each slot of s_buf
    __shared__ uint32_t s_tot[kW];
    __shared__ int s_map[MAP ? 3 * kMaxViews : 1];
    const int64_t n = live_count(n_max, n_dev);
    const int64_t start = (int64_t)blockIdx.x * kTileN;
    if (start >= n) return;                                  // uniform across the block
    const int count = (int)min((int64_t)kTileN, n - start);
    const int lane = __lane_id(), wid = threadIdx.x >> 6;
    const int t = threadIdx.x;                               // digit of the per-digit phases (t < 256)
    const uint64_t lt = lanemask_lt();
    if constexpr (MAP) {
        if (t == 0) rows.stage(s_map);                       // read after the barriers below
    }
#pragma unroll
    for (int k = 0; k < kRadixBins / 64; ++k) s_wc[wid][lane + 64 * k] = 0u;
    {
        // global base of digit t: all smaller digits + this digit in earlier blocks
        const uint32_t tot = t < kRadixBins ? digit_total[t] : 0u;
        uint32_t all;
        const uint32_t before = block_exclusive_scan<uint32_t, kW>(tot, all, s_tot);
        if (t < kRadixBins) s_gbase[t] = before + hist_scan[(int64_t)t * stride + blockIdx.x];
    }

    const KT *kin = keys_in + start;                        // uniform bases, 32-bit offsets
    const uint32_t *vin = vals_in ? vals_in + start : nullptr;
    uint32_t key[ITEMS], lp[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const int local = wid * kPerWave + r * 64 + lane;
        key[r] = local < count ? (uint32_t)kin[local] : 0u;
    }
    // item r takes part: in the block, and (first planned pass with a drop)
    // not culled; the other instantiations test the block bound alone
    uint32_t livem = 0u;
    if constexpr (PLAN) {
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) {
            const int local = wid * kPerWave + r * 64 + lane;
            livem |= (local < count && ds.keep(key[r]) ? 1u : 0u) << r;
        }
    }
    auto live = [&](int r) -> bool {
        if constexpr (PLAN) return (livem >> r) & 1u;
        else return wid * kPerWave + r * 64 + lane < count;
    };
    if (ds.rebase) {                                        // after the loads: all of them in flight at once
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) key[r] = ds.key(key[r]);
    }
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const bool active = live(r);
        const uint32_t d = (key[r] >> ds.shift) & ds.mask;
        const uint64_t match = digit_match(active, d, ds.nbits);
        const uint32_t before = active ? s_wc[wid][d] : 0u;
        const uint32_t within = (uint32_t)__popcll(match & lt);
        lp[r] = before + within;                             // rank within the wavefront's digit run
        if (active && within == 0) s_wc[wid][d] = before + (uint32_t)__popcll(match);
        wave_sync_lds();
    }
    __syncthreads();
    // digit t: prefix over wavefronts, block total, exclusive scan over digits
    uint32_t ntot;
    {
        uint32_t run = 0;
        if (t < kRadixBins) {
#pragma unroll
            for (int w = 0; w < kW; ++w) {
                const uint32_t c = s_wc[w][t];
                s_wc[w][t] = run;
                run += c;
            }
        }
        const uint32_t ex = block_exclusive_scan<uint32_t, kW>(run, ntot, s_tot);
        if (t < kRadixBins) s_lbase[t] = ex;
    }
    // elements staged in digit order: all of the block's, or its kept ones
    const int placed = PLAN ? (int)ntot : count;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        if (live(r)) {
            const uint32_t d = (key[r] >> ds.shift) & ds.mask;
            lp[r] += s_lbase[d] + s_wc[wid][d];
            s_buf[lp[r]] = key[r];
            s_dig[lp[r]] = (uint8_t)d;
        }
    }
    // values travel in the second half: load them now, while the keys are
    // written out
    uint32_t val[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const int local = wid * kPerWave + r * 64 + lane;
        val[r] = local < count ? (vin ? vin[local] : (uint32_t)(start + local)) : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const int i = threadIdx.x + r * NT;
        if (i < placed) {
            const uint32_t d = s_dig[i];
            const uint32_t k = s_buf[i];
            keys_out[s_gbase[d] + (uint32_t)i - s_lbase[d]] = MAP ? rows.tile_of(k, s_map) : k;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        if (live(r)) s_buf[lp[r]] = val[r];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const int i = threadIdx.x + r * NT;
        if (i < placed) {
            const uint32_t d = s_dig[i];
            const uint32_t pos = s_gbase[d] + (uint32_t)i - s_lbase[d];
            const uint32_t v = s_buf[i];
            vals_out[pos] = v;
            // optional: carry the 16-byte record of element v to its sorted place
            if (gather_dst) gather_dst[pos] = gather_src[v];
        }
    }
    if (aux.out) {
        // the third payload through the same LDS buffer
        uint32_t x[ITEMS];
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) {
            const int local = wid * kPerWave + r * 64 + lane;
            x[r] = local < count ? (aux.in ? aux.in[start + local] : pack_rect(aux.pack[start + local])) : 0u;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) {
            if (live(r)) s_buf[lp[r]] = x[r];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) {
            const int i = threadIdx.x + r * NT;
            if (i < placed) {
                const uint32_t d = s_dig[i];
                aux.out[s_gbase[d] + (uint32_t)i - s_lbase[d]] = s_buf[i];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Column-first binning (views at most 256 tiles wide).  Tile ids are ordered
// by (view, tile row, tile column), so a stable pass by tile column followed
// by a stable sort by global tile row (the rows of all views stacked) leaves
// every tile's pairs in depth order.  The column pass needs no pair list in
// memory: the pairs a block of Gaussians puts into column c number the sum
// of the row spans of its rectangles that cover c (a difference array over
// the columns), and the pairs themselves are generated from the rectangles
// while they are placed.  This replaces the duplication and the first radix
// pass over the pairs.  Keys in between: (global row << 8) | column.
// ---------------------------------------------------------------------------
constexpr int kColBits = 8;
constexpr int kMaxCols = 1 << kColBits;            // tiles per view row
constexpr int kColBlock = 512;                     // Gaussians per column block (= scatter threads)
constexpr int kColItems = 4;                       // pairs per thread and chunk
static_assert(kMaxCols == kRadixBins && kMaxCols == kBlock, "one column per digit and per thread");

// rectangle columns clamped to [0, kMaxCols] (a no-op for projected
// rectangles, which lie inside their view's grid)
__device__ __forceinline__ int4 col_rect(int4 q)
{
    q.x = min(max(q.x, 0), kMaxCols);
    q.z = min(max(q.z, q.x), kMaxCols);
    return q;
}

// Rectangle reader of the column pass: int4 records (columns clamped) or
// packed ones.
struct RectInt4 {
    const int4 *p;
    __device__ __forceinline__ int4 operator()(int64_t i) const { return col_rect(p[i]); }
};
struct RectPacked {
    const uint32_t *p;
    __device__ __forceinline__ int4 operator()(int64_t i) const { return unpack_rect(p[i]); }
};

// Exact tile assignment.  A splat's tiles are those of its rectangle whose
// pixel-centre square [16 col, 16 col + 15] x [16 row, 16 row + 15] its
// alpha >= 1/255 ellipse meets (the tile assignment of Sec. II-A made exact,
// as in the block-level culling the paper composes with).  Per tile column,
// the ellipse's vertical span over the column's pixel-centre range (the
// render's tight-box test of Sec. III-C-2 on the same enlarged ellipse, so the
// set is a superset of the exact one) gives the rows it meets.  The column
// histogram counts with this function and the scatter tests its candidates
// with it; the file is built without floating-point contraction so that both
// take every decision alike.
struct Splat {
    float mx, my, a, b, c, lo;
};

__device__ __forceinline__ Splat load_splat(const float *__restrict__ splats, uint32_t g)
{
    const float4 *rec = splat_rec(splats, g);
    const float4 k = rec[0], m = rec[1];
    return Splat{m.x, m.y, k.x, k.y, k.z, __builtin_amdgcn_logf(k.w)};
}

// tile rows [x, y] (view-local, unclipped; empty when x > y) of tile column
// `col` that the splat's ellipse meets
__device__ __forceinline__ int2 exact_rows(const Splat &g, int col)
{
    float ymin, ymax;
    const float x0 = (float)(col * kTile) - g.mx, x1 = x0 + (float)(kTile - 1);
    if (!render::column_span(g.a, g.b, g.c, g.lo, x0, x1, ymin, ymax)) return make_int2(1, 0);
    // row r meets when 16 r <= my + ymax and 16 r + 15 >= my + ymin (1e-3 px slack)
    const float top = fminf(fmaxf(g.my + ymin - 1e-3f, -1e8f), 1e8f);
    const float bot = fminf(fmaxf(g.my + ymax + 1e-3f, -1e8f), 1e8f);
    return make_int2((int)ceilf((top - (float)(kTile - 1)) * (1.0f / kTile)), (int)floorf(bot * (1.0f / kTile)));
}

// geometry of the splats (view-major element ids), or none: rectangles only
struct SplatGeom {
    const float *splats;
};

// Per-block column counts: hist[c * stride + b] = pairs of column c among the
// Gaussians [b * kColBlock, (b + 1) * kColBlock) of the depth order.  One
// workgroup counts kHistGroup consecutive blocks (one 16-byte write per
// column) and writes their pair total to block_pairs[workgroup].
template <typename RIN, bool EXACT>
__global__ __launch_bounds__(kBlock) void col_hist_kernel(const RIN rect, int64_t n_max, const uint32_t *n_dev,
                                                          int ncols, uint32_t *__restrict__ hist, int64_t stride,
                                                          uint64_t *__restrict__ block_pairs,
                                                          const uint32_t *__restrict__ order, SplatGeom geom)
{
    const int64_t n = live_count(n_max, n_dev);              // Gaussians in the depth order
    __shared__ uint32_t s_d[kMaxCols + 1];
    __shared__ uint32_t s_warp[kWaves];
    __shared__ uint64_t s_pairs[kHistGroup];
    const int t = threadIdx.x;
    if (t < kHistGroup) s_pairs[t] = 0ull;
    uint32_t c[kHistGroup];
#pragma unroll
    for (int j = 0; j < kHistGroup; ++j) {
        s_d[t] = 0u;
        if (t == 0) s_d[kMaxCols] = 0u;
        __syncthreads();
        const int64_t r0 = ((int64_t)blockIdx.x * kHistGroup + j) * kColBlock;
        uint64_t pairs = 0;
#pragma unroll
        for (int i = 0; i < kColBlock / kBlock; ++i) {
            const int64_t r = r0 + i * kBlock + t;
            if (r < n) {
                const int4 q = rect(r);
                if (q.z > q.x && q.w > q.y) {
                    if constexpr (EXACT) {
                        // each column its own row count: a difference pair per column
                        const Splat sp = load_splat(geom.splats, order[r]);
                        for (int col = q.x; col < q.z; ++col) {
                            const int2 rr = exact_rows(sp, col);
                            const int h = min(rr.y, q.w - 1) - max(rr.x, q.y) + 1;
                            if (h > 0) {
                                atomicAdd(&s_d[col], (uint32_t)h);
                                atomicAdd(&s_d[col + 1], 0u - (uint32_t)h);
                                pairs += (uint64_t)h;
                            }
                        }
                    } else {
                        const uint32_t h = (uint32_t)(q.w - q.y);
                        atomicAdd(&s_d[q.x], h);
                        atomicAdd(&s_d[q.z], 0u - h);
                        pairs += (uint64_t)h * (uint64_t)(q.z - q.x);
                    }
                }
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) pairs += __shfl_xor(pairs, off, 64);
        if (__lane_id() == 0) atomicAdd(&s_pairs[j], pairs);
        __syncthreads();
        uint32_t tot;
        const uint32_t d = s_d[t];
        c[j] = block_exclusive_scan<uint32_t, kWaves>(d, tot, s_warp) + d;
    }
    if (t < ncols)
        *reinterpret_cast<uint4 *>(hist + (int64_t)t * stride + (int64_t)blockIdx.x * kHistGroup) =
            make_uint4(c[0], c[1], c[2], c[3]);
    if (t == 0) {
        uint64_t sum = 0;
#pragma unroll
        for (int j = 0; j < kHistGroup; ++j) sum += s_pairs[j];
        block_pairs[blockIdx.x] = sum;
    }
}

// Scan of the per-block column counts (workgroup c < ncols: column c, as a
// radix row scan) and, in the extra last workgroup, the total pair count P
// (64-bit sum of the block totals), the overflow flag and min(P, capacity).
struct PairTotal {
    const uint64_t *block_pairs;
    int64_t nb;
    uint64_t cap;
    uint64_t *total_out;
    int64_t *num_pairs;
    int32_t *overflow;
    uint32_t *n_eff;
};

__global__ __launch_bounds__(kBlock) void col_rowscan_kernel(uint32_t *__restrict__ hist, int64_t stride, int64_t n,
                                                             int ncols, uint32_t *__restrict__ col_total,
                                                             PairTotal pt)
{
    if ((int)blockIdx.x < ncols) {
        radix_rowscan_body<32>(hist, stride, n, nullptr, kColBlock, col_total);
        return;
    }
    __shared__ uint64_t s_warp[kWaves];
    constexpr int kU = 16;                                 // independent loads in flight per thread
    uint64_t sum = 0;
    for (int64_t i0 = threadIdx.x; i0 < pt.nb; i0 += (int64_t)kBlock * kU) {
        uint64_t part[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int64_t i = i0 + (int64_t)u * kBlock;
            part[u] = i < pt.nb ? pt.block_pairs[i] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) sum += part[u];
    }
    uint64_t total;
    block_exclusive_scan<uint64_t, kWaves>(sum, total, s_warp);
    if (threadIdx.x == 0) {
        *pt.total_out = total;
        *pt.num_pairs = (int64_t)total;
        *pt.overflow = total > pt.cap ? 1 : 0;
        *pt.n_eff = (uint32_t)(total > pt.cap ? pt.cap : total);
    }
}

// Generation and column placement of the pairs of one block of kColBlock
// Gaussians, in chunks of kColBlock * ITEMS pairs.  Per chunk: every thread
// generates ITEMS consecutive pairs of the block's depth-ordered, row-major
// enumeration (one binary search over the block's pair offsets, then
// stepping through the rectangle) into LDS; the wavefronts rank them by
// column in that enumeration order (so a column keeps depth order, and row
// order within a Gaussian); the chunk is then ordered by column in LDS (key
// and owning Gaussian) and each column run is written to its place: the
// column's global start plus the column's pairs in earlier blocks and in
// earlier chunks of this one.  Places at or past the capacity are not
// written.
template <int ITEMS, typename KT, typename RIN, bool EXACT>
__global__ __launch_bounds__(kColBlock) void col_scatter_kernel(
    const uint32_t *__restrict__ order, const RIN rect, uint64_t cap, TileGrids tg, int64_t n_max,
    const uint32_t *n_dev,
    const uint32_t *__restrict__ hist_scan, const uint32_t *__restrict__ col_total, int64_t stride, int ncols,
    int nbits, KT *__restrict__ keys_out, uint32_t *__restrict__ vals_out, SplatGeom geom)
{
    constexpr int NT = kColBlock;
    constexpr int kW = NT / 64;
    constexpr int kTileN = NT * ITEMS;
    constexpr int kPerWave = kTileN / kW;
    static_assert(ITEMS % 4 == 0, "16-byte staging writes");
    __shared__ uint32_t s_xw[NT];                          // first column | width << 16
    __shared__ uint32_t s_id[NT];
    __shared__ uint32_t s_row[NT];                         // global tile row of the rectangle's first row
    __shared__ uint32_t s_off[NT + 1];                     // block-local r-major pair offsets
    __shared__ uint32_t s_gb[2][kMaxCols];                 // per chunk parity: global place of its column runs
    __shared__ uint32_t s_wc[kW][kMaxCols];
    __shared__ uint32_t s_lbase[kMaxCols];
    __shared__ __align__(16) uint32_t s_buf[kTileN];       // generated keys, then keys by column
    __shared__ __align__(16) uint16_t s_own[kTileN];       // block-local Gaussian of each generated pair
    __shared__ uint16_t s_osort[kTileN];                   // the same, by column
    __shared__ uint32_t s_tot[kW];
    // exact assignment: the block's splats and the first (view-local) row of
    // each rectangle; a candidate tile of the rectangle is generated only if
    // its row is among those the splat meets in its column
    __shared__ Splat s_sp[EXACT ? NT : 1];
    __shared__ int s_y0[EXACT ? NT : 1];
    constexpr uint32_t kNone = 0xFFFFFFFFu;                // key of a candidate the ellipse misses
    const int64_t n = live_count(n_max, n_dev);              // Gaussians in the depth order
    const int64_t first = (int64_t)blockIdx.x * NT;
    if (first >= n) return;
    const int cnt = (int)min((int64_t)NT, n - first);
    const int t = threadIdx.x, lane = __lane_id(), wid = t >> 6;
    const uint64_t lt = lanemask_lt();
    const uint32_t dmask = (1u << nbits) - 1u;              // columns < 2^nbits
    uint32_t npairs = 0;
    if (t < cnt) {
        const uint32_t g = order[first + t];
        const int v = tg.V > 1 ? (int)(g / tg.per_view) : 0;
        const int4 q = rect(first + t);
        const bool has = q.z > q.x && q.w > q.y;
        s_xw[t] = (uint32_t)q.x | ((uint32_t)(q.z - q.x) << 16);
        s_id[t] = g;
        s_row[t] = (uint32_t)(tg.row_off[v] + q.y);
        npairs = has ? (uint32_t)(q.z - q.x) * (uint32_t)(q.w - q.y) : 0u;
        if constexpr (EXACT) {
            if (has) s_sp[t] = load_splat(geom.splats, g);
            s_y0[t] = q.y;
        }
    }
    {
        // block-local r-major offsets of the Gaussians' pairs
        uint32_t all;
        const uint32_t ex = block_exclusive_scan<uint32_t, kW>(npairs, all, s_tot);
        s_off[t] = ex;
        if (t == NT - 1) s_off[NT] = all;
    }
    {
        // global start of column t (exclusive scan of the column totals) plus
        // the column's pairs in earlier blocks
        const uint32_t tot = t < ncols ? col_total[t] : 0u;
        uint32_t all;
        const uint32_t before = block_exclusive_scan<uint32_t, kW>(tot, all, s_tot);
        if (t < kMaxCols) s_gb[0][t] = before + (t < ncols ? hist_scan[(int64_t)t * stride + blockIdx.x] : 0u);
    }
    __syncthreads();
    const uint32_t m = s_off[NT];                           // pairs of this block
    int par = 0;
    for (uint32_t q0 = 0; q0 < m; q0 += kTileN, par ^= 1) {
        const int count = (int)min((uint32_t)kTileN, m - q0);
        // 1. generate ITEMS consecutive pairs per thread (blocked layout)
        {
            const uint32_t p0 = q0 + (uint32_t)t * ITEMS;
            uint32_t kk[ITEMS], ow[ITEMS];
#pragma unroll
            for (int e = 0; e < ITEMS; ++e) { kk[e] = 0u; ow[e] = 0u; }
            if (p0 < m) {
                int lo = 0, hi = cnt - 1;                   // last k with s_off[k] <= p0
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (s_off[mid] <= p0) lo = mid; else hi = mid - 1;
                }
                int k = lo;
                uint32_t nx = s_off[k + 1];                 // end of Gaussian k's pairs
                uint32_t xw = s_xw[k], row = s_row[k];
                uint32_t w = xw >> 16;
                const uint32_t i = p0 - s_off[k];
                uint32_t ty = w ? i / w : 0u, tx = i - ty * w;
#pragma unroll
                for (int e = 0; e < ITEMS; ++e) {
                    const uint32_t p = p0 + e;
                    if (p < m) {
                        while (p >= nx) {                   // next Gaussian that has pairs
                            ++k;
                            nx = s_off[k + 1];
                            xw = s_xw[k];
                            row = s_row[k];
                            w = xw >> 16;
                            tx = 0;
                            ty = 0;
                        }
                        const uint32_t col = (xw & 0xFFFFu) + tx;
                        kk[e] = ((row + ty) << kColBits) | col;
                        if constexpr (EXACT) {
                            const int2 rr = exact_rows(s_sp[k], (int)col);
                            const int r = s_y0[k] + (int)ty;
                            if (r < rr.x || r > rr.y) kk[e] = kNone;
                        }
                        ow[e] = (uint32_t)k;
                        if (++tx == w) { tx = 0; ++ty; }
                    }
                }
            }
            uint4 *b4 = reinterpret_cast<uint4 *>(s_buf + t * ITEMS);
#pragma unroll
            for (int e = 0; e < ITEMS; e += 4) b4[e / 4] = make_uint4(kk[e], kk[e + 1], kk[e + 2], kk[e + 3]);
            uint2 *o2 = reinterpret_cast<uint2 *>(s_own + t * ITEMS);
#pragma unroll
            for (int e = 0; e < ITEMS; e += 4)
                o2[e / 4] = make_uint2(ow[e] | (ow[e + 1] << 16), ow[e + 2] | (ow[e + 3] << 16));
        }
#pragma unroll
        for (int k = 0; k < kMaxCols / 64; ++k) s_wc[wid][lane + 64 * k] = 0u;
        __syncthreads();
        // 2. rank by column, rounds of 64 consecutive pairs per wavefront
        uint32_t key[ITEMS], lp[ITEMS];
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) key[r] = s_buf[wid * kPerWave + r * 64 + lane];
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) {
            // a chunk is often far from full (a block of Gaussians averages
            // fewer pairs than a chunk holds): rounds past its end are empty,
            // and so are all later ones
            if (__builtin_amdgcn_readfirstlane(wid * kPerWave + r * 64) >= count) break;
            const int local = wid * kPerWave + r * 64 + lane;
            const bool active = local < count && (!EXACT || key[r] != kNone);
            const uint32_t d = key[r] & dmask;
            const uint64_t match = digit_match(active, d, nbits);
            const uint32_t before = active ? s_wc[wid][d] : 0u;
            const uint32_t within = (uint32_t)__popcll(match & lt);
            lp[r] = before + within;
            if (active && within == 0) s_wc[wid][d] = before + (uint32_t)__popcll(match);
            wave_sync_lds();
        }
        __syncthreads();
        // 3. per column: prefix over wavefronts, chunk offsets, next chunk's bases
        uint32_t placed;                                      // pairs of this chunk (candidates kept)
        {
            uint32_t ccount = 0;
            if (t < kMaxCols) {
#pragma unroll
                for (int w = 0; w < kW; ++w) {
                    const uint32_t c = s_wc[w][t];
                    s_wc[w][t] = ccount;
                    ccount += c;
                }
                s_gb[par ^ 1][t] = s_gb[par][t] + ccount;
            }
            const uint32_t ex = block_exclusive_scan<uint32_t, kW>(ccount, placed, s_tot);
            if (t < kMaxCols) s_lbase[t] = ex;
        }
        __syncthreads();
        // 4. order the chunk by column in LDS
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) {
            const int local = wid * kPerWave + r * 64 + lane;
            if (local < count && (!EXACT || key[r] != kNone)) {
                const uint32_t d = key[r] & dmask;
                const uint32_t at = lp[r] + s_lbase[d] + s_wc[wid][d];
                s_buf[at] = key[r];
                s_osort[at] = s_own[local];
            }
        }
        __syncthreads();
        // 5. write the column runs (consecutive lanes, consecutive places)
        const uint32_t *gb = s_gb[par];
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) {
            const int i = t + r * NT;
            if (i < (int)placed) {
                const uint32_t k = s_buf[i];
                const uint32_t d = k & dmask;
                const uint32_t pos = gb[d] + (uint32_t)i - s_lbase[d];
                if (pos < cap) {
                    keys_out[pos] = (KT)k;                  // 16-bit keys: rows and columns below 256
                    vals_out[pos] = s_id[s_osort[i]];
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// tile ranges: 4 sorted keys per lane, vector loads.  Every tile is written
// once: a run's start and end at the key changes, and the tiles between two
// runs (and before the first and after the last) as empty (0, 0), so no
// clearing pass is needed.  With an overflow or no pairs all tiles are empty.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void zero_tiles(uint2 *ranges, uint32_t a, uint32_t b)
{
    for (uint32_t t = a; t < b; ++t) ranges[t] = make_uint2(0u, 0u);
}

__global__ void ranges_kernel(const uint32_t *__restrict__ keys, const int64_t *num_pairs, const int32_t *overflow,
                              int64_t cap, uint32_t num_tiles, uint2 *__restrict__ ranges)
{
    int64_t n = *num_pairs;
    if (n > cap) n = cap;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if ((overflow && *overflow) || n <= 0) {
        for (int64_t t = tid; t < num_tiles; t += (int64_t)gridDim.x * blockDim.x) ranges[t] = make_uint2(0u, 0u);
        return;
    }
    const int64_t stride = (int64_t)gridDim.x * blockDim.x * 4;
    for (int64_t i0 = tid * 4; i0 < n; i0 += stride) {
        uint32_t k[5];
        if (i0 + 3 < n && ((reinterpret_cast<uintptr_t>(keys + i0) & 15) == 0)) {
            const uint4 v = *reinterpret_cast<const uint4 *>(keys + i0);
            k[0] = v.x; k[1] = v.y; k[2] = v.z; k[3] = v.w;
        } else {
            for (int e = 0; e < 4; ++e) k[e] = i0 + e < n ? keys[i0 + e] : 0xFFFFFFFFu;
        }
        k[4] = i0 + 4 < n ? keys[i0 + 4] : 0xFFFFFFFFu;
        uint32_t prev = i0 > 0 ? keys[i0 - 1] : 0xFFFFFFFFu;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t i = i0 + e;
            if (i < n && k[e] < num_tiles) {                  // keys of valid input always are
                if (i == 0) {
                    zero_tiles(ranges, 0u, k[e]);
                    ranges[k[e]].x = 0u;
                } else if (prev != k[e]) {
                    ranges[k[e]].x = (uint32_t)i;
                    if (prev < k[e]) zero_tiles(ranges, prev + 1u, k[e]);
                }
                if (i + 1 >= n) {
                    ranges[k[e]].y = (uint32_t)n;
                    zero_tiles(ranges, k[e] + 1u, num_tiles);
                } else if (k[e + 1] != k[e]) {
                    ranges[k[e]].y = (uint32_t)(i + 1);
                }
            }
            prev = k[e];
        }
    }
}

// Work-order key of a tile for longest-first scheduling: 255 minus a
// logarithmic code of its list length with 8 steps per octave, so one stable
// 8-bit pass orders the tiles by non-increasing length class, index order
// within a class.  Empty tiles get key 255.
__global__ void lpt_key_kernel(const uint2 *__restrict__ ranges, int64_t num_tiles, uint32_t *__restrict__ keys)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= num_tiles) return;
    const uint2 r = ranges[t];
    const uint32_t len = r.y > r.x ? r.y - r.x : 0u;
    uint32_t code = 0;
    if (len > 0) {
        const uint32_t e = 31u - (uint32_t)__clz(len);
        const uint32_t m = e >= 3 ? (len >> (e - 3)) & 7u : (len << (3 - e)) & 7u;
        code = min(e * 8u + m + 1u, 255u);
    }
    keys[t] = 255u - code;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
inline size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

struct SortWorkspace {
    uint32_t *dk[2], *dv[2];      // depth keys / ids, ping-pong [n]
    uint32_t *pk, *pv;            // alternate pair buffers [cap]
    uint32_t *hist;               // [256 * nblocks_max]
    uint32_t *digit_total;        // [256]
    uint32_t *pair_off;           // [n] pair counts, then exclusive offsets
    int4 *rect_sorted;            // [n] tile rectangles in depth order
    uint64_t *partials;           // scan partials
    uint64_t *col_pairs;          // pair total of each column block
    uint32_t *n_eff;              // min(P, cap)
    uint64_t *p_total;            // P
    uint32_t *range;              // [lo, hi, count] of the visible depth keys
    uint4 *range_parts;           // per-workgroup extremes and counts of the range's first step
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
    // per-block counts of the radix passes and of the column pass
    const int64_t nb_radix = hist_stride(radix_blocks(n > cap ? n : cap) + 1);
    const int64_t nb_col = hist_stride((nm + kColBlock - 1) / kColBlock + 1);
    const int64_t nbmax = nb_radix > nb_col ? nb_radix : nb_col;
    w.hist = (uint32_t *)take(sizeof(uint32_t) * kRadixBins * nbmax);
    w.digit_total = (uint32_t *)take(sizeof(uint32_t) * kRadixBins);
    w.pair_off = (uint32_t *)take(sizeof(uint32_t) * nm);
    w.rect_sorted = (int4 *)take(sizeof(int4) * nm);
    w.partials = (uint64_t *)take(sizeof(uint64_t) * ((nm + kScanTile - 1) / kScanTile + 1));
    w.col_pairs = (uint64_t *)take(sizeof(uint64_t) * nb_col);
    w.n_eff = (uint32_t *)take(sizeof(uint32_t));
    w.p_total = (uint64_t *)take(sizeof(uint64_t));
    w.range = (uint32_t *)take(4 * sizeof(uint32_t));
    w.range_parts = (uint4 *)take(kRangeParts * sizeof(uint4));
    w.bytes = off;
    return w;
}

// one stable radix pass over [0, min(n_max, *n_dev)) on key bits
// [shift, shift + bits)
template <int ITEMS, int SCATTER_THREADS, typename KT>
void radix_pass_t(const KT *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout, int64_t n_max,
                  const uint32_t *n_dev, int shift, int bits, const SortWorkspace &w, hipStream_t s,
                  const int4 *gather_src, int4 *gather_dst, const RowMap &rows, const AuxPayload &aux, bool top,
                  const DepthPlan &dp)
{
    constexpr int kTileN = kBlock * ITEMS;
    const int64_t nb = (n_max + kTileN - 1) / kTileN;
    if (nb == 0) return;
    const int64_t stride = hist_stride(nb);
    // bank-staggered counter copies where digits repeat within a wavefront:
    // the top digit of a key, and long inputs (sorted pairs, stacked views)
    // few blocks (short inputs): one block per workgroup, so that more of the
    // chip counts; else kHistGroup blocks per workgroup and 16-byte writes
    const bool copies = top || ITEMS >= 16, few = nb < 2048;
    const dim3 hg((unsigned)(few ? nb : stride / kHistGroup));
    constexpr int kScatterItems = ITEMS * kBlock / SCATTER_THREADS;   // same partition as the histogram
    // the depth passes with a digit plan are instantiated apart, so that the
    // others compile exactly as without one
    auto launch = [&](auto plan) {
        constexpr bool P = decltype(plan)::value;
        if (copies && few)
            hipLaunchKernelGGL((radix_hist_kernel<ITEMS, KT, 4, 1, P>), hg, dim3(kBlock), 0, s, kin, n_max, n_dev,
                               shift, bits, w.hist, stride, dp);
        else if (copies)
            hipLaunchKernelGGL((radix_hist_kernel<ITEMS, KT, 4, kHistGroup, P>), hg, dim3(kBlock), 0, s, kin, n_max,
                               n_dev, shift, bits, w.hist, stride, dp);
        else if (few)
            hipLaunchKernelGGL((radix_hist_kernel<ITEMS, KT, 1, 1, P>), hg, dim3(kBlock), 0, s, kin, n_max, n_dev,
                               shift, bits, w.hist, stride, dp);
        else
            hipLaunchKernelGGL((radix_hist_kernel<ITEMS, KT, 1, kHistGroup, P>), hg, dim3(kBlock), 0, s, kin, n_max,
                               n_dev, shift, bits, w.hist, stride, dp);
        hipLaunchKernelGGL(radix_rowscan_kernel, dim3(kRadixBins), dim3(kBlock), 0, s, w.hist, stride, n_max, n_dev,
                           kTileN, w.digit_total);
        if constexpr (!P) {
            if (rows.V) {
                hipLaunchKernelGGL((radix_scatter_kernel<kScatterItems, SCATTER_THREADS, true, KT, false>),
                                   dim3((unsigned)nb), dim3(SCATTER_THREADS), 0, s, kin, vin, kout, vout, n_max, n_dev,
                                   shift, bits, (const uint32_t *)w.hist, (const uint32_t *)w.digit_total, stride,
                                   gather_src, gather_dst, rows, aux, dp);
                return;
            }
        }
        hipLaunchKernelGGL((radix_scatter_kernel<kScatterItems, SCATTER_THREADS, false, KT, P>), dim3((unsigned)nb),
                           dim3(SCATTER_THREADS), 0, s, kin, vin, kout, vout, n_max, n_dev, shift, bits,
                           (const uint32_t *)w.hist, (const uint32_t *)w.digit_total, stride, gather_src, gather_dst,
                           rows, aux, dp);
    };
    if (dp.range)
        launch(std::true_type{});
    else
        launch(std::false_type{});
}

template <typename KT>
void radix_pass(const KT *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout, int64_t n_max,
                const uint32_t *n_dev, int shift, int bits, const SortWorkspace &w, hipStream_t s,
                const int4 *gather_src = nullptr, int4 *gather_dst = nullptr, const RowMap &rows = RowMap{},
                const AuxPayload &aux = AuxPayload{}, bool top = false, const DepthPlan &dp = DepthPlan{})
{
    if (n_max >= kLargeRadixFrom)
        radix_pass_t<32, 1024>(kin, vin, kout, vout, n_max, n_dev, shift, bits, w, s, gather_src, gather_dst, rows,
                               aux, top, dp);
    else
        radix_pass_t<kRadixItems, 1024>(kin, vin, kout, vout, n_max, n_dev, shift, bits, w, s, gather_src,
                                        gather_dst, rows, aux, top, dp);
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

extern "C" lgs_status lgs_sort_batch(int32_t num_views, const int32_t *tiles_x, const int32_t *tiles_y,
                                     int64_t n_per_view, const float *depth, const int32_t *rect,
                                     const float *splats, uint32_t *tile_keys, uint32_t *values,
                                     int64_t capacity_pairs,
                                     int64_t *num_pairs, int32_t *overflow, void *workspace, size_t workspace_bytes,
                                     void *stream)
{
    LGS_REQUIRE(num_views >= 1 && num_views <= kMaxViews && tiles_x && tiles_y,
                "lgs_sort: num_views must be 1..%d with tile grids", kMaxViews);
    LGS_REQUIRE(n_per_view >= 0 && n_per_view * num_views < (int64_t)UINT32_MAX, "lgs_sort: n out of range");
    const int64_t n = n_per_view * num_views;
    TileGrids tg{};
    tg.per_view = (uint32_t)(n_per_view > 0 ? n_per_view : 1);
    tg.V = num_views;
    int64_t total_tiles = 0, total_rows = 0;
    int ncols = 0, nrows = 0;
    RowMap rows{};
    rows.V = num_views;
    for (int v = 0; v < num_views; ++v) {
        LGS_REQUIRE(tiles_x[v] > 0 && tiles_y[v] > 0, "lgs_sort: bad tile grid of view %d", v);
        tg.tile_off[v] = (int)total_tiles;
        tg.tiles_x[v] = tiles_x[v];
        tg.row_off[v] = (int)total_rows;
        rows.row_off[v] = (int)total_rows;
        rows.tiles_x[v] = tiles_x[v];
        rows.base[v] = (int)(total_tiles - total_rows * tiles_x[v]);
        total_tiles += (int64_t)tiles_x[v] * tiles_y[v];
        total_rows += tiles_y[v];
        ncols = tiles_x[v] > ncols ? tiles_x[v] : ncols;
        nrows = tiles_y[v] > nrows ? tiles_y[v] : nrows;
        LGS_REQUIRE(total_tiles < (1ll << 31), "lgs_sort: too many tiles");
    }
    LGS_REQUIRE(capacity_pairs >= 0 && capacity_pairs < (int64_t)UINT32_MAX, "lgs_sort: capacity out of range");
    LGS_REQUIRE(num_pairs && overflow, "lgs_sort: null num_pairs/overflow");
    LGS_REQUIRE(n == 0 || (depth && rect), "lgs_sort: null input");
    LGS_REQUIRE(capacity_pairs == 0 || (tile_keys && values), "lgs_sort: null output");
    LGS_REQUIRE(((uintptr_t)tile_keys % 16 == 0) && ((uintptr_t)values % 16 == 0),
                "lgs_sort: tile_keys and values must be 16-byte aligned");
    LGS_REQUIRE(rect == nullptr || (uintptr_t)rect % 16 == 0, "lgs_sort: rect must be 16-byte aligned");
    LGS_REQUIRE((uintptr_t)splats % 16 == 0, "lgs_sort: splats must be 16-byte aligned");
    const size_t need = plan_workspace(nullptr, n, capacity_pairs).bytes;
    LGS_REQUIRE(workspace && workspace_bytes >= need, "lgs_sort: workspace too small (%zu < %zu bytes)",
                workspace_bytes, need);
    LGS_REQUIRE((uintptr_t)workspace % 256 == 0, "lgs_sort: workspace must be 256-byte aligned");
    hipStream_t s = as_stream(stream);
    SortWorkspace w = plan_workspace(static_cast<char *>(workspace), n, capacity_pairs);
    const int4 *rc = reinterpret_cast<const int4 *>(rect);

    // Column-first binning (views up to kMaxCols tiles wide) sorts by the
    // global tile row after its column pass; otherwise the pairs are
    // duplicated and sorted by tile id.  With views at most 256 tiles high as
    // well, the rectangles travel packed in 32 bits.
    const bool by_column = ncols <= kMaxCols;
    const bool packed = by_column && nrows <= 256;
    // exact tile assignment on the column path (grids at most 256 tiles wide)
    const bool exact = by_column && splats != nullptr;
    const SplatGeom geom{splats};
    uint32_t *rp[2] = {reinterpret_cast<uint32_t *>(w.rect_sorted), reinterpret_cast<uint32_t *>(w.rect_sorted) + n};

    // 1. stable sort of all Gaussians by depth bits (positive floats order
    //    like their bit patterns; culled ones hold +inf and end up last):
    //    the range of the visible keys, then four passes over the bits in
    //    which they differ (the digit plan above), the first reading the
    //    depths and implicit ids.  The rectangles follow into depth order:
    //    packed, as a payload of every pass (the first packs them from the
    //    input, in index order), or else gathered by the last pass.
    const uint32_t *dbits = reinterpret_cast<const uint32_t *>(depth);
    // the plan from 2^20 Gaussians up; below, its two extra launches cost more
    // than the narrower digits save, and the passes take 8 bits each
    const bool plan = n >= kPlanFrom;
    if (plan) {
        const int nparts = (int)min((unsigned)kRangeParts, grid_for(n, 4 * kBlock));
        hipLaunchKernelGGL(depth_range_kernel, dim3((unsigned)nparts), dim3(kBlock), 0, s, dbits, n, w.range_parts);
        hipLaunchKernelGGL(depth_range_final_kernel, dim3(1), dim3(kRangeParts), 0, s, (const uint4 *)w.range_parts,
                           nparts, w.range);
    }
    // on the column path the planned first pass also leaves the culled
    // Gaussians out: the later passes and the column pass take the visible
    // count (culled ones have no tiles, and nothing else reads their place)
    const bool drop = plan && by_column;
    const uint32_t *n_vis = drop ? w.range + 2 : nullptr;
    {
        AuxPayload aux{};
        if (packed) {
            aux.out = rp[0];
            aux.pack = rc;
        }
        radix_pass(dbits, nullptr, w.dk[0], w.dv[0], n, nullptr, 0, 8, w, s, nullptr, nullptr, RowMap{}, aux, false,
                   DepthPlan{plan ? w.range : nullptr, 0, drop});
    }
    for (int pass = 1; pass < 4; ++pass) {
        const int a = (pass - 1) & 1;
        AuxPayload aux{};
        if (packed) {
            aux.in = rp[a];
            aux.out = rp[a ^ 1];
        }
        const bool gather = !packed && pass == 3;
        radix_pass(w.dk[a], w.dv[a], w.dk[a ^ 1], w.dv[a ^ 1], n, n_vis, 8 * pass, 8, w, s,
                   gather ? rc : nullptr, gather ? w.rect_sorted : nullptr, RowMap{}, aux, pass == 3,
                   DepthPlan{plan ? w.range : nullptr, pass, false});
    }
    const uint32_t *order = w.dv[1];          // passes 0..3 leave the result in buffer 1
    const RectPacked rect_packed{rp[1]};
    const RectInt4 rect_int4{w.rect_sorted};
    // 2. The number of tile-sort passes decides which buffer receives the
    //    pairs so that the sorted result ends in the caller's.
    // with fewer than 256 global rows the keys between the column and the row
    // pass fit 16 bits (row << 8 | column), and the row pass is a single one
    const bool key16 = by_column && total_rows <= 256;
    int bits = 1;
    while ((1ll << bits) < (by_column ? total_rows : total_tiles)) ++bits;
    const int passes = (bits + kRadixBits - 1) / kRadixBits;
    uint32_t *k0 = (passes & 1) ? w.pk : tile_keys, *v0 = (passes & 1) ? w.pv : values;
    uint32_t *k1 = (passes & 1) ? tile_keys : w.pk, *v1 = (passes & 1) ? values : w.pv;
    if (by_column) {
        // 3. column pass: per-block column counts (and pair totals, whose sum
        //    is P), their scan per column, and generation + placement of the
        //    pairs
        const int64_t nbc = (n + kColBlock - 1) / kColBlock;
        const int64_t stride = hist_stride(nbc);
        int cbits = 1;
        while ((1 << cbits) < ncols) ++cbits;
        const dim3 hgrid((unsigned)(stride / kHistGroup));
        if (n > 0 && packed && exact)
            hipLaunchKernelGGL((col_hist_kernel<RectPacked, true>), hgrid, dim3(kBlock), 0, s, rect_packed, n, n_vis, ncols,
                               w.hist, stride, w.col_pairs, order, geom);
        else if (n > 0 && packed)
            hipLaunchKernelGGL((col_hist_kernel<RectPacked, false>), hgrid, dim3(kBlock), 0, s, rect_packed, n, n_vis, ncols,
                               w.hist, stride, w.col_pairs, order, geom);
        else if (n > 0 && exact)
            hipLaunchKernelGGL((col_hist_kernel<RectInt4, true>), hgrid, dim3(kBlock), 0, s, rect_int4, n, n_vis, ncols,
                               w.hist, stride, w.col_pairs, order, geom);
        else if (n > 0)
            hipLaunchKernelGGL((col_hist_kernel<RectInt4, false>), hgrid, dim3(kBlock), 0, s, rect_int4, n, n_vis, ncols,
                               w.hist, stride, w.col_pairs, order, geom);
        const int64_t nhg = n > 0 ? stride / kHistGroup : 0;      // column-histogram workgroups
        const PairTotal pt{w.col_pairs, nhg, (uint64_t)capacity_pairs, w.p_total, num_pairs, overflow, w.n_eff};
        hipLaunchKernelGGL(col_rowscan_kernel, dim3(n > 0 ? ncols + 1 : 1), dim3(kBlock), 0, s, w.hist, stride, n,
                           n > 0 ? ncols : 0, w.digit_total, pt);
        const uint32_t *hs = w.hist, *ct = w.digit_total;
        const uint64_t cp = (uint64_t)capacity_pairs;
        const dim3 sgrid((unsigned)nbc), sblk(kColBlock);
        uint16_t *k16 = reinterpret_cast<uint16_t *>(k0);
        if (n > 0 && key16 && exact)                          // 16-bit keys imply packed rectangles
            hipLaunchKernelGGL((col_scatter_kernel<kColItems, uint16_t, RectPacked, true>), sgrid, sblk, 0, s, order,
                               rect_packed, cp, tg, n, n_vis, hs, ct, stride, ncols, cbits, k16, v0, geom);
        else if (n > 0 && key16)
            hipLaunchKernelGGL((col_scatter_kernel<kColItems, uint16_t, RectPacked, false>), sgrid, sblk, 0, s, order,
                               rect_packed, cp, tg, n, n_vis, hs, ct, stride, ncols, cbits, k16, v0, geom);
        else if (n > 0 && packed && exact)
            hipLaunchKernelGGL((col_scatter_kernel<kColItems, uint32_t, RectPacked, true>), sgrid, sblk, 0, s, order,
                               rect_packed, cp, tg, n, n_vis, hs, ct, stride, ncols, cbits, k0, v0, geom);
        else if (n > 0 && packed)
            hipLaunchKernelGGL((col_scatter_kernel<kColItems, uint32_t, RectPacked, false>), sgrid, sblk, 0, s, order,
                               rect_packed, cp, tg, n, n_vis, hs, ct, stride, ncols, cbits, k0, v0, geom);
        else if (n > 0 && exact)
            hipLaunchKernelGGL((col_scatter_kernel<kColItems, uint32_t, RectInt4, true>), sgrid, sblk, 0, s, order,
                               rect_int4, cp, tg, n, n_vis, hs, ct, stride, ncols, cbits, k0, v0, geom);
        else if (n > 0)
            hipLaunchKernelGGL((col_scatter_kernel<kColItems, uint32_t, RectInt4, false>), sgrid, sblk, 0, s, order,
                               rect_int4, cp, tg, n, n_vis, hs, ct, stride, ncols, cbits, k0, v0, geom);
    } else {
        // 3. pair counts in depth order, their exclusive scan (total P,
        //    overflow) and duplication in depth order
        const int64_t nb = (n + kScanTile - 1) / kScanTile;
        if (nb > 0)
            hipLaunchKernelGGL((scan_reduce_kernel<uint64_t, PairCountGather>), dim3((unsigned)nb), dim3(kBlock), 0,
                               s, PairCountGather{w.rect_sorted, w.pair_off}, n, (const uint32_t *)nullptr,
                               w.partials);
        hipLaunchKernelGGL(pair_partials_kernel, dim3(1), dim3(1024), 0, s, w.partials, nb, w.p_total,
                           (uint64_t)capacity_pairs, num_pairs, overflow, w.n_eff);
        if (nb > 0)
            hipLaunchKernelGGL((scan_final_kernel<uint64_t, U32Load, OffsetStore>), dim3((unsigned)nb), dim3(kBlock),
                               0, s, U32Load{w.pair_off}, OffsetStore{w.pair_off, (uint64_t)capacity_pairs}, n,
                               (const uint32_t *)nullptr, (const uint64_t *)w.partials);
        if (n > 0)
            hipLaunchKernelGGL(duplicate_kernel, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, order,
                               (const int4 *)w.rect_sorted, (const uint32_t *)w.pair_off,
                               (const uint64_t *)w.p_total, (uint64_t)capacity_pairs, tg, n, k0, v0);
    }
    // 4. stable sort of the pairs by global tile row (above the column bits,
    //    the last pass writing tile ids) or by tile id, the key bits split
    //    evenly over the passes (longer digit runs per block than 8 + remainder)
    const int base_shift = by_column ? kColBits : 0;
    if (key16) {
        radix_pass(reinterpret_cast<const uint16_t *>(k0), v0, k1, v1, capacity_pairs, w.n_eff, kColBits, bits, w, s,
                   nullptr, nullptr, rows, AuxPayload{}, true);
    } else {
        for (int pass = 0, shift = 0; pass < passes; ++pass) {
            const int b = (bits - shift + (passes - pass) - 1) / (passes - pass);
            const RowMap map = by_column && pass == passes - 1 ? rows : RowMap{};
            const bool top = pass == passes - 1;
            if (pass & 1)
                radix_pass(k1, v1, k0, v0, capacity_pairs, w.n_eff, base_shift + shift, b, w, s, nullptr, nullptr, map,
                           AuxPayload{}, top);
            else
                radix_pass(k0, v0, k1, v1, capacity_pairs, w.n_eff, base_shift + shift, b, w, s, nullptr, nullptr, map,
                           AuxPayload{}, top);
            shift += b;
        }
    }
    LGS_LAUNCHED("lgs_sort");
    return LGS_OK;
}

extern "C" lgs_status lgs_sort(int64_t n, int32_t tiles_x, int32_t tiles_y, const float *depth, const int32_t *rect,
                               const float *splats, uint32_t *tile_keys, uint32_t *values, int64_t capacity_pairs,
                               int64_t *num_pairs, int32_t *overflow, void *workspace, size_t workspace_bytes,
                               void *stream)
{
    return lgs_sort_batch(1, &tiles_x, &tiles_y, n, depth, rect, splats, tile_keys, values,
                          capacity_pairs, num_pairs, overflow, workspace, workspace_bytes, stream);
}

// ---------------------------------------------------------------------------
// lgs_sort_noalloc: lgs_sort on the library's own scratch.  The scratch is a
// file-scope device array; in host code its name is not a device address, so
// the address is looked up with hipGetSymbolAddress once per device (on the
// first call with that device current) and only that address is passed on.
// Every call on a device shares its array.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[LGS_SORT_NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[64] = {};
}  // namespace

extern "C" lgs_status lgs_sort_noalloc(int64_t n, int32_t tiles_x, int32_t tiles_y, const float *depth,
                                       const int32_t *rect, const float *splats, uint32_t *tile_keys,
                                       uint32_t *values, int64_t capacity_pairs,
                                       int64_t *num_pairs, int32_t *overflow, void *stream)
{
    LGS_REQUIRE(n >= 0 && capacity_pairs >= 0, "lgs_sort_noalloc: n and capacity_pairs must be >= 0");
    const size_t need = plan_workspace(nullptr, n, capacity_pairs).bytes;
    LGS_REQUIRE(need <= (size_t)LGS_SORT_NOALLOC_SCRATCH_BYTES,
                "lgs_sort_noalloc: %lld Gaussians with a capacity of %lld pairs need %zu bytes of scratch, more "
                "than the library's %zu; use lgs_sort with a workspace of lgs_sort_workspace_size() bytes",
                (long long)n, (long long)capacity_pairs, need, (size_t)LGS_SORT_NOALLOC_SCRATCH_BYTES);
    int dev = -1;
    LGS_HIP(hipGetDevice(&dev));
    LGS_REQUIRE(dev >= 0 && dev < 64, "lgs_sort_noalloc: device index %d out of range", dev);
    void *ptr = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (g_scratch_ptr[dev] == nullptr) {
            void *p = nullptr;
            const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            LGS_REQUIRE(e == hipSuccess && p != nullptr, "lgs_sort_noalloc: scratch address on device %d: %s", dev,
                        hipGetErrorString(e));
            g_scratch_ptr[dev] = p;
        }
        ptr = g_scratch_ptr[dev];
    }
    return lgs_sort_batch(1, &tiles_x, &tiles_y, n, depth, rect, splats, tile_keys, values,
                          capacity_pairs, num_pairs, overflow, ptr, (size_t)LGS_SORT_NOALLOC_SCRATCH_BYTES, stream);
}

extern "C" lgs_status lgs_tile_ranges(const uint32_t *tile_keys, const int64_t *num_pairs, const int32_t *overflow,
                                      int64_t capacity_pairs, int32_t num_tiles, uint32_t *ranges, void *stream)
{
    LGS_REQUIRE(num_tiles > 0 && ranges && num_pairs, "lgs_tile_ranges: bad arguments");
    LGS_REQUIRE(capacity_pairs >= 0 && (capacity_pairs == 0 || tile_keys), "lgs_tile_ranges: bad pair buffer");
    LGS_REQUIRE((uintptr_t)ranges % 8 == 0, "lgs_tile_ranges: ranges must be 8-byte aligned");
    hipStream_t s = as_stream(stream);
    const int64_t work = capacity_pairs / 4 > num_tiles ? capacity_pairs / 4 : num_tiles;
    unsigned g = grid_for(work, 256);
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(ranges_kernel, dim3(g), dim3(256), 0, s, tile_keys, num_pairs, overflow, capacity_pairs,
                       (uint32_t)num_tiles, reinterpret_cast<uint2 *>(ranges));
    LGS_LAUNCHED("lgs_tile_ranges");
    return LGS_OK;
}

namespace {
struct OrderWorkspace {
    uint32_t *keys, *keys_out, *hist, *digit_total;
    size_t bytes;
};

OrderWorkspace plan_order(char *base, int64_t num_tiles)
{
    OrderWorkspace w{};
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off += align_up(bytes > 0 ? bytes : 1);
        return p;
    };
    w.keys = (uint32_t *)take(sizeof(uint32_t) * num_tiles);
    w.keys_out = (uint32_t *)take(sizeof(uint32_t) * num_tiles);
    w.hist = (uint32_t *)take(sizeof(uint32_t) * kRadixBins * hist_stride(radix_blocks(num_tiles) + 1));
    w.digit_total = (uint32_t *)take(sizeof(uint32_t) * kRadixBins);
    w.bytes = off;
    return w;
}
}  // namespace

extern "C" size_t lgs_tile_order_workspace_size(int32_t num_tiles)
{
    if (num_tiles <= 0) return 0;
    return plan_order(nullptr, num_tiles).bytes;
}

extern "C" lgs_status lgs_tile_order(const uint32_t *ranges, int32_t num_tiles, uint32_t *order, void *workspace,
                                     size_t workspace_bytes, void *stream)
{
    LGS_REQUIRE(num_tiles > 0 && ranges && order, "lgs_tile_order: bad arguments");
    LGS_REQUIRE((uintptr_t)ranges % 8 == 0, "lgs_tile_order: ranges must be 8-byte aligned");
    const OrderWorkspace need = plan_order(nullptr, num_tiles);
    LGS_REQUIRE(workspace && workspace_bytes >= need.bytes && (uintptr_t)workspace % 256 == 0,
                "lgs_tile_order: workspace must be 256-byte aligned and at least %zu bytes", need.bytes);
    hipStream_t s = as_stream(stream);
    const OrderWorkspace ow = plan_order(static_cast<char *>(workspace), num_tiles);
    hipLaunchKernelGGL(lpt_key_kernel, dim3(grid_for(num_tiles, 256)), dim3(256), 0, s,
                       reinterpret_cast<const uint2 *>(ranges), (int64_t)num_tiles, ow.keys);
    SortWorkspace w{};
    w.hist = ow.hist;
    w.digit_total = ow.digit_total;
    radix_pass(ow.keys, nullptr, ow.keys_out, order, num_tiles, nullptr, 0, 8, w, s);
    LGS_LAUNCHED("lgs_tile_order");
    return LGS_OK;
}
