// Render kernel: front-to-back alpha blending of each 16x16 tile, with the
// three Local-GS stages re-derived for 64-lane wavefronts (Sec. III).
//
// One workgroup of 256 lanes per tile; wavefront w covers the 16x4 pixel
// strip of rows 4w..4w+3 (the paper uses 16x2 strips for 32-lane warps,
// Sec. III-C-1).
//
// Variants (cumulative ablation ladder of the paper):
//   PLAIN       baseline loop (Alg. 1, baseline column): the workgroup stages
//               batches of 256 list entries in LDS; every lane evaluates the
//               quadratic in screen coordinates, skips below 1/255 and breaks
//               at T < 1e-4 on its own.
//   HOIST       + tile-local hoisting (Sec. III-B): staging computes
//               V = H(delta) [a, b, c, log2 o] once per (tile, Gaussian); each
//               lane evaluates the exponent as a 5-FMA dot product with its
//               fixed basis [x'^2, x'y', y'^2, x', y', 1].
//   HOIST_CULL  + wavefront culling before prefetching (Sec. III-C): each
//               wavefront walks the list in chunks of 64 on its own, tests its
//               16x4 strip against the tight vertical span of the footprint
//               (cases A/B/C), and hoists only the surviving entries into a
//               dense per-wavefront LDS list.  Blending keeps the per-lane
//               skip and break of the baseline.
//   LOCAL       + uniform blending (Sec. III-D): the same staging; the blend is
//               branch-free (alpha zeroed by a select in the log2 domain,
//               w = alpha T, C += c w, T -= w under a per-lane live predicate)
//               and the wavefront stops on a ballot vote.
//
// Precision.  With R = double the exponent (the hoisted dot product, or the
// plain quadratic) is evaluated in double, which gfx950 issues at the FP32
// rate, so the expanded tile-local polynomial carries no cancellation error
// and every variant obtains the same float32 exponent; alpha, T and the
// colour are float, and every variant updates T <- fma(-alpha, T, T), so
// the ladder reproduces the plain renderer up to rare float32 rounding flips
// of the exponent.  R = float is the paper's single-precision arithmetic
// throughout, with its literal updates: T (1 - alpha) in the per-pixel loops
// and T - w in the uniform blend.  The exponential itself is v_exp_f32 of a
// float32 log2-domain exponent in every variant.
#include "common.hpp"

#include "render_common.hpp"

namespace lgs {
namespace {

using namespace render;

// the paper's literal single-precision updates (R = float) or the fused one
template <typename R>
constexpr bool kLiteral = sizeof(R) == 4;

// ---------------------------------------------------------------------------
// PLAIN and HOIST: workgroup-cooperative batches (the baseline structure)
// ---------------------------------------------------------------------------
struct PlainEntry {       // screen-space mean, conic, log2 opacity (or opacity)
    float mx, my, a, b, c, lo;
};

template <bool HOISTED, typename R, bool STATS>
__global__ __launch_bounds__(kBlock) void render_block_kernel(RenderArgs args)
{
    using Entry = typename std::conditional<HOISTED, Hoisted<R>, PlainEntry>::type;
    __shared__ Entry s_e[kBlock];
    __shared__ float4 s_c[kBlock];
    __shared__ int s_alive[kBlock / 64];

    const TileCtx<R> tc(args, args.order ? (int)args.order[blockIdx.x] : xcd_tile(blockIdx.x, args.num_tiles),
                        threadIdx.x >> 6);
    float T = 1.f;
    float C0 = 0.f, C1 = 0.f, C2 = 0.f;
    int32_t last = 0;
    bool done = !tc.inside;
    unsigned long long st_seen = 0, st_eval = 0, st_staged = 0;
    const uint2 range = args.ranges[tc.tile];

    for (uint32_t base = range.x; base < range.y; base += kBlock) {
        // workgroup-wide vote: stop fetching once every pixel has terminated
        const bool any = __ballot(!done) != 0ull;
        if (__lane_id() == 0) s_alive[tc.wid] = any;
        __syncthreads();
        if (!(s_alive[0] | s_alive[1] | s_alive[2] | s_alive[3])) break;
        const int nb = (int)min((uint32_t)kBlock, range.y - base);

        // cooperative staging: one list entry per lane
        if ((int)threadIdx.x < nb) {
            const uint32_t g = args.values[base + threadIdx.x];
            const float4 *rec = splat_rec(args.splats, g);
            const float4 co = rec[0], mr = rec[1];
            const float2 m = make_float2(mr.x, mr.y);
            const float lo = __builtin_amdgcn_logf(co.w);   // v_log_f32 (log2)
            s_c[threadIdx.x] = make_float4(mr.z, mr.w, reinterpret_cast<const float *>(rec + 2)[0], 0.f);
            if constexpr (HOISTED) {
                s_e[threadIdx.x] = hoist<R>(m, co, lo, tc.ox, tc.oy);
            } else {
                PlainEntry e;
                e.mx = m.x; e.my = m.y; e.a = co.x; e.b = co.y; e.c = co.z;
                e.lo = sizeof(R) == 8 ? lo : co.w;
                s_e[threadIdx.x] = e;
            }
        }
        if (STATS) st_staged += nb;
        __syncthreads();

        for (int j = 0; j < nb; ++j) {
            if (done) break;
            if (STATS) { st_seen++; st_eval++; }
            const float4 f = s_c[j];
            float al;
            bool keep;
            if constexpr (HOISTED) {
                const float s32 = (float)dot_exponent(s_e[j], tc);
                al = fminf(__builtin_amdgcn_exp2f(s32), kAlphaMax);
                keep = s32 >= kLog2AlphaMin;
            } else {
                const PlainEntry e = s_e[j];
                if constexpr (sizeof(R) == 8) {
                    const double dx = (double)tc.px - (double)e.mx, dy = (double)tc.py - (double)e.my;
                    const double q = (double)e.a * dx * dx + 2.0 * (double)e.b * dx * dy + (double)e.c * dy * dy;
                    const float s32 = (float)((double)e.lo - 0.5 * kLog2e * q);
                    al = fminf(__builtin_amdgcn_exp2f(s32), kAlphaMax);
                    keep = s32 >= kLog2AlphaMin;
                } else {
                    // the 3DGS expression, in float
                    const float dx = e.mx - (float)tc.px, dy = e.my - (float)tc.py;
                    const float power = -0.5f * (e.a * dx * dx + e.c * dy * dy) - e.b * dx * dy;
                    al = fminf(e.lo * __builtin_amdgcn_exp2f(power * (float)kLog2e), kAlphaMax);
                    keep = al >= kAlphaMinF;
                }
            }
            if (!keep) continue;
            const float test = kLiteral<R> ? T * (1.f - al) : fmaf(-al, T, T);
            if (test < (float)kTMin) { done = true; break; }
            const float w = al * T;
            C0 = fmaf(f.x, w, C0);
            C1 = fmaf(f.y, w, C1);
            C2 = fmaf(f.z, w, C2);
            T = test;
            last = (int32_t)(base + j - range.x + 1);
        }
    }
    write_pixel(args, tc, C0, C1, C2, T, last);
    if (STATS) flush_stats<false>(args, st_seen, st_eval, st_staged);
}

// ---------------------------------------------------------------------------
// HOIST_CULL and LOCAL: wavefront-autonomous, culling before prefetching
// ---------------------------------------------------------------------------
struct WaveStats {
    unsigned long long seen = 0, eval = 0, staged = 0;
};

// one lane's list entry of a chunk: its splat record's fields (a culled or
// past-the-end lane holds a zero-size placeholder that no test keeps)
struct ChunkEntry {
    float4 co;              // a, b, c, o
    float4 mr;              // x, y, r, g
    float b;
};

__device__ __forceinline__ ChunkEntry load_entry(const RenderArgs &a, uint32_t id, bool valid)
{
    ChunkEntry e{make_float4(0.f, 0.f, 0.f, 1.f), make_float4(0.f, 0.f, 0.f, 0.f), 0.f};
    if (valid) {
        const float4 *rec = splat_rec(a.splats, id);
        e.co = rec[0];
        e.mr = rec[1];
        e.b = reinterpret_cast<const float *>(rec + 2)[0];
    }
    return e;
}

// One 16x4 strip of one tile, processed by one wavefront with its own LDS
// slots (no workgroup barrier).  MASKS: record the used-entry masks (a
// forward that a backward follows); a forward without them saves the per-step
// compare and its scalar bookkeeping.
template <bool UNIFORM, typename R, bool STATS, int VP, bool MASKS>
__device__ __forceinline__ void render_strip(const RenderArgs &args, const TileCtx<R> &tc, Hoisted<R> *s_e,
                                             float4 *s_c, WaveStats &st)
{
    float T = 1.f;
    float C0 = 0.f, C1 = 0.f, C2 = 0.f;
    int32_t last = 0;
    bool live = tc.inside;
    const uint2 range = args.ranges[tc.tile];
    const uint64_t lt = lanemask_lt();
    // this wavefront's sub-tile: columns [sx0, sx1], rows [sy0, sy1]
    const int sx0 = tc.sx0, sx1 = tc.sx1, sy0 = tc.sy0, sy1 = tc.sy1;
    bool wave_live = __ballot(live) != 0ull;

    // Two-deep software pipeline over the chunks: while chunk i is culled and
    // blended, the records of chunk i + 1 (by ids already in registers) and
    // the ids of chunk i + 2 are in flight.
    // (positions in 64 bits: no wrap near the end of a 32-bit pair range)
    const uint32_t lane = __lane_id();
    const uint64_t end = range.y;
    auto load_id = [&](uint64_t b) -> uint32_t { return b + lane < end ? args.values[b + lane] : 0u; };
    ChunkEntry nxt = load_entry(args, load_id(range.x), (uint64_t)range.x + lane < end);
    uint32_t id_next = load_id((uint64_t)range.x + 64);

    for (uint64_t base64 = range.x; wave_live && base64 < end; base64 += 64) {
        const uint32_t base = (uint32_t)base64;
        const uint32_t j = base + lane;
        const ChunkEntry cur = nxt;
        nxt = load_entry(args, id_next, base64 + 64 + lane < end);
        id_next = load_id(base64 + 128);
        bool hit = false;
        const float4 co = cur.co;
        const float2 m = make_float2(cur.mr.x, cur.mr.y);
        float lo = 0.f;
        const bool in_list = base64 + lane < end;
        if (in_list) {
            lo = __builtin_amdgcn_logf(co.w);
            hit = strip_hit(co.x, co.y, co.z, lo, (float)sx0 - m.x, (float)sx1 - m.x, (float)sy0 - m.y,
                            (float)sy1 - m.y);
        }
        const uint64_t bits = __ballot(hit);
        const int cnt = __popcll(bits);
        if (STATS) st.staged += cnt;
        // culling record: this wavefront tested entry j (bit w) and kept it (bit 4 + w)
        if (STATS && args.masks != nullptr && in_list)
            atomicOr(&args.masks[j], (1u << tc.wid) | (hit ? (16u << tc.wid) : 0u));
        if (hit) {
            const int slot = __popcll(bits & lt);
            s_e[slot] = hoist<R>(m, co, lo, tc.ox, tc.oy);
            s_c[slot] = make_float4(cur.mr.z, cur.mr.w, cur.b, __int_as_float((int)(j - range.x + 1)));
        }
        if (UNIFORM && VP > 1) {
            // pad the list to a multiple of VP with entries that no pixel
            // keeps (log2 alpha = -inf; position -1, never a last
            // contributor), so that the unrolled steps need no exit test
            const int padded = (cnt + VP - 1) / VP * VP;
            if ((int)lane >= cnt && (int)lane < padded) {
                Hoisted<R> z;
#pragma unroll
                for (int c = 0; c < 5; ++c) z.v[c] = (R)0;
                z.v[5] = (R)(-INFINITY);
                s_e[lane] = z;
                s_c[lane] = make_float4(0.f, 0.f, 0.f, __int_as_float(-1));
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        const int chunk = (int)min((uint32_t)64, range.y - base);
        int consumed = chunk;
        uint64_t used = 0;              // staged slots that some lane of the wavefront blended
        if constexpr (UNIFORM) {
            // the wave-wide vote runs once per VP Gaussians; steps after the
            // last lane has stopped change nothing (every update is masked by
            // the lane's live predicate)
            for (int k0 = 0; k0 < cnt; k0 += VP) {
                int kdone = k0;
#pragma unroll
                for (int u = 0; u < VP; ++u) {
                const int k = k0 + u;
                if (VP == 1) kdone = k;
                else if (k < cnt) kdone = k;
                const float4 f = s_c[k];
                const float s32 = (float)dot_exponent(s_e[k], tc);
                const bool keep = s32 >= kLog2AlphaMin;
                const float alpha = keep ? fminf(__builtin_amdgcn_exp2f(s32), kAlphaMax) : 0.f;
                const float w = alpha * T;
                const float Tn = kLiteral<R> ? T - w : fmaf(-alpha, T, T);
                const bool lv = live && !(Tn < (float)kTMin);
                const float wl = lv ? w : 0.f;
                C0 = fmaf(f.x, wl, C0);
                C1 = fmaf(f.y, wl, C1);
                C2 = fmaf(f.z, wl, C2);
                T = lv ? Tn : T;
                last = (lv && keep) ? __float_as_int(f.w) : last;
                live = lv;
                // lanes that blended this Gaussian: exactly those whose last
                // contributor is now this list position (one compare, mask in
                // scalar registers)
                if constexpr (MASKS) {
                    if (__builtin_amdgcn_uicmp((uint32_t)last, (uint32_t)__float_as_int(f.w), 32) != 0ull)
                        used |= 1ull << k;
                }
                if (STATS && k < cnt) st.eval++;
                }
                if (__builtin_amdgcn_ballot_w64(live) == 0ull) {
                    wave_live = false;
                    if (STATS) consumed = __float_as_int(s_c[kdone].w) - (int)(base - range.x);
                    break;
                }
            }
        } else {
            bool done = !live;
            int lane_evals = 0;
            for (int k = 0; k < cnt; ++k) {
                if (done) break;
                if (STATS) lane_evals++;
                const float4 f = s_c[k];
                const float s32 = (float)dot_exponent(s_e[k], tc);
                const float al = fminf(__builtin_amdgcn_exp2f(s32), kAlphaMax);
                if (!(s32 >= kLog2AlphaMin)) continue;
                const float test = kLiteral<R> ? T * (1.f - al) : fmaf(-al, T, T);
                if (test < (float)kTMin) { done = true; break; }
                const float w = al * T;
                C0 = fmaf(f.x, w, C0);
                C1 = fmaf(f.y, w, C1);
                C2 = fmaf(f.z, w, C2);
                T = test;
                last = __float_as_int(f.w);
            }
            live = !done;
            if (STATS) {
                int mx = lane_evals;
                for (int off = 32; off > 0; off >>= 1) mx = max(mx, __shfl_xor(mx, off, 64));
                st.eval += mx;
            }
            wave_live = __ballot(live) != 0ull;
        }
        if constexpr (UNIFORM && MASKS) {
            // record, by list position, the chunk's entries that some lane
            // of this sub-tile blended (the entries its backward replays)
            const uint64_t pos_used = __ballot(hit && ((used >> __popcll(bits & lt)) & 1ull));
            const int64_t wd = used_word(range.x, tc.tile, base);
            if (lane == 0 && wd < args.used_plane) args.used[(int64_t)tc.wid * args.used_plane + wd] = pos_used;
        }
        if (STATS) st.seen += consumed;
        // all lanes have read this chunk before the next one overwrites it
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    write_pixel(args, tc, C0, C1, C2, T, last);
}

// Grid mode: workgroup = tile, wavefront = strip.  Persistent mode
// (args.queue != null): every wavefront pops (tile, strip) units from a
// device counter until all 4 * num_tiles units are taken, so no wavefront
// waits for the others of its workgroup and the tail is balanced.  There is
// one counter per XCD (workgroups are dispatched round-robin over the 8
// XCDs, so workgroup b draws from counter b % 8, each on its own cache
// line): counter x hands out the four strips of queue positions x, x + 8,
// x + 16, ..., which spreads the atomics over eight addresses and keeps the
// strips of one tile within one XCD's L2.
// (at least four wavefronts per SIMD: the allocator otherwise lets a variant
// grow a few registers past 128 and lose a quarter of its occupancy)
template <bool UNIFORM, typename R, bool STATS, bool Q8, int VP, bool MASKS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void render_wave_kernel(RenderArgs args)
{
    __shared__ Hoisted<R> s_e[kBlock / 64][64];
    __shared__ float4 s_c[kBlock / 64][64];        // colour, list position in .w
    const int wid = threadIdx.x >> 6;
    WaveStats st;
    if (args.queue == nullptr) {
        const TileCtx<R> tc(args, args.order ? (int)args.order[blockIdx.x] : xcd_tile(blockIdx.x, args.num_tiles),
                            wid, Q8);
        render_strip<UNIFORM, R, STATS, VP, MASKS>(args, tc, s_e[wid], s_c[wid], st);
    } else {
        const uint32_t units = 4u * (uint32_t)args.num_tiles;
        const uint32_t x = blockIdx.x & (kQueues - 1);
        uint32_t *counter = args.queue + x * kQueueStride;
        for (;;) {
            uint32_t j = 0;
            if (__lane_id() == 0) j = atomicAdd(counter, 1u);
            j = __builtin_amdgcn_readfirstlane(j);
            const uint64_t u64 = (uint64_t)(j >> 2) * (4u * kQueues) + 4u * x + (j & 3u);
            if (u64 >= units) break;
            const uint32_t u = (uint32_t)u64;
            const int tile = args.order ? (int)args.order[u >> 2] : (int)(u >> 2);
            const TileCtx<R> tc(args, tile, (int)(u & 3u), Q8);
            render_strip<UNIFORM, R, STATS, VP, MASKS>(args, tc, s_e[wid], s_c[wid], st);
        }
    }
    if (STATS) flush_stats<true>(args, st.seen, st.eval, st.staged);
}

template <bool UNIFORM, typename R, bool Q8, int VP>
void launch_wave(bool stats, dim3 g, dim3 block, hipStream_t s, const RenderArgs &a)
{
    if (UNIFORM && a.used != nullptr) {
        if (stats) hipLaunchKernelGGL((render_wave_kernel<UNIFORM, R, true, Q8, VP, UNIFORM>), g, block, 0, s, a);
        else hipLaunchKernelGGL((render_wave_kernel<UNIFORM, R, false, Q8, VP, UNIFORM>), g, block, 0, s, a);
    } else {
        if (stats) hipLaunchKernelGGL((render_wave_kernel<UNIFORM, R, true, Q8, VP, false>), g, block, 0, s, a);
        else hipLaunchKernelGGL((render_wave_kernel<UNIFORM, R, false, Q8, VP, false>), g, block, 0, s, a);
    }
}

template <int V, typename R>
void launch_render(const RenderArgs &a, bool stats, bool q8, bool vote4, unsigned grid, hipStream_t s)
{
    const dim3 g(grid), block(kBlock);
    switch (V) {
    case LGS_RENDER_PLAIN:
        if (stats) hipLaunchKernelGGL((render_block_kernel<false, R, true>), g, block, 0, s, a);
        else hipLaunchKernelGGL((render_block_kernel<false, R, false>), g, block, 0, s, a);
        break;
    case LGS_RENDER_HOIST:
        if (stats) hipLaunchKernelGGL((render_block_kernel<true, R, true>), g, block, 0, s, a);
        else hipLaunchKernelGGL((render_block_kernel<true, R, false>), g, block, 0, s, a);
        break;
    case LGS_RENDER_HOIST_CULL:
        if (q8) launch_wave<false, R, true, 1>(stats, g, block, s, a);
        else launch_wave<false, R, false, 1>(stats, g, block, s, a);
        break;
    default:
        if (vote4) {
            if (q8) launch_wave<true, R, true, 4>(stats, g, block, s, a);
            else launch_wave<true, R, false, 4>(stats, g, block, s, a);
        } else {
            if (q8) launch_wave<true, R, true, 1>(stats, g, block, s, a);
            else launch_wave<true, R, false, 1>(stats, g, block, s, a);
        }
        break;
    }
}

}  // namespace
}  // namespace lgs

using namespace lgs;

namespace {
lgs_status render_batch(int32_t variant, const lgs_camera *cameras, int32_t num_views, const uint32_t *ranges,
                        const uint32_t *values, const float *splats, float *out_rgb, float *out_T,
                        int32_t *out_ncontrib, uint64_t *stats, uint32_t *queue,
                        const uint32_t *tile_order, int32_t blocks_per_cu, uint32_t *masks, uint64_t *used_masks,
                        int64_t used_mask_words, void *stream)
{
    LGS_REQUIRE(num_views >= 1 && num_views <= kMaxViews, "lgs_render_batch: num_views must be 1..%d",
                kMaxViews);
    LGS_REQUIRE(cameras != nullptr, "lgs_render_batch: null cameras");
    Cam cams[kMaxViews];
    for (int v = 0; v < num_views; ++v)
        LGS_REQUIRE(cam_from(&cameras[v], cams[v]), "lgs_render_batch: invalid camera %d", v);
    const int v = variant & 0xF;
    const bool fp32 = (variant & LGS_RENDER_FP32) != 0;
    const bool q8 = (variant & LGS_RENDER_Q8) != 0;
    const bool vote4 = (variant & LGS_RENDER_VOTE4) != 0;
    LGS_REQUIRE(v >= 0 && v <= 3
                    && (variant & ~(0xF | LGS_RENDER_FP32 | LGS_RENDER_Q8 | LGS_RENDER_VOTE4 | LGS_RENDER_GLOBAL)) == 0,
                "lgs_render: unknown variant %d", variant);
    LGS_REQUIRE(ranges && out_rgb && out_T && out_ncontrib, "lgs_render: null argument");
    LGS_REQUIRE(((uintptr_t)ranges % 8 == 0) && ((uintptr_t)splats % 16 == 0),
                "lgs_render: ranges must be 8-byte and splats 16-byte aligned");
    LGS_REQUIRE(used_masks == nullptr || (used_mask_words >= 4 && (uintptr_t)used_masks % 8 == 0),
                "lgs_render_batch: used_masks needs 8-byte alignment and at least 4 words");
    render::RenderArgs a = render::make_args(cams, num_views, ranges, values, splats, out_rgb, out_T, out_ncontrib,
                                             stats);
    hipStream_t s = as_stream(stream);
    a.order = tile_order;                     // queue position -> tile, or workgroup -> tile
    a.global_origin = (variant & LGS_RENDER_GLOBAL) != 0;
    a.masks = masks;
    a.used = used_masks;
    a.used_plane = used_masks ? used_mask_words / 4 : 0;
    const bool persistent = queue != nullptr && (v == LGS_RENDER_HOIST_CULL || v == LGS_RENDER_LOCAL);
    unsigned grid = (unsigned)a.num_tiles;
    if (persistent) {
        static_assert(kQueues * kQueueStride == LGS_QUEUE_WORDS, "queue block size");
        fill_async<uint32_t>(queue, 0u, kQueues * kQueueStride, s);
        a.queue = queue;
        const int per = blocks_per_cu > 0 ? blocks_per_cu : 8;
        // a multiple of kQueues, so that every counter has workgroups taking from it
        grid = (unsigned)((device_cus() * per + kQueues - 1) / kQueues * kQueues);
    }
    const bool st = stats != nullptr;
    if (fp32) {
        switch (v) {
        case 0: launch_render<0, float>(a, st, q8, vote4, grid, s); break;
        case 1: launch_render<1, float>(a, st, q8, vote4, grid, s); break;
        case 2: launch_render<2, float>(a, st, q8, vote4, grid, s); break;
        default: launch_render<3, float>(a, st, q8, vote4, grid, s); break;
        }
    } else {
        switch (v) {
        case 0: launch_render<0, double>(a, st, q8, vote4, grid, s); break;
        case 1: launch_render<1, double>(a, st, q8, vote4, grid, s); break;
        case 2: launch_render<2, double>(a, st, q8, vote4, grid, s); break;
        default: launch_render<3, double>(a, st, q8, vote4, grid, s); break;
        }
    }
    LGS_LAUNCHED("lgs_render");
    return LGS_OK;
}
}  // namespace

extern "C" lgs_status lgs_render_batch(int32_t variant, const lgs_camera *cameras, int32_t num_views,
                                       const uint32_t *ranges, const uint32_t *values, const float *splats,
                                       float *out_rgb, float *out_T, int32_t *out_ncontrib, uint64_t *stats,
                                       uint32_t *queue, const uint32_t *tile_order, int32_t blocks_per_cu,
                                       uint64_t *used_masks, int64_t used_mask_words, void *stream)
{
    return render_batch(variant, cameras, num_views, ranges, values, splats, out_rgb, out_T, out_ncontrib, stats,
                        queue, tile_order, blocks_per_cu, nullptr, used_masks, used_mask_words, stream);
}

extern "C" int64_t lgs_used_mask_words(int64_t capacity_pairs, int32_t num_tiles)
{
    if (capacity_pairs < 0 || num_tiles < 0) return 0;
    return 4 * ((capacity_pairs >> 6) + (int64_t)num_tiles + 1);
}

extern "C" lgs_status lgs_render_debug(int32_t variant, const lgs_camera *cameras, int32_t num_views,
                                       const uint32_t *ranges, const uint32_t *values, const float *splats,
                                       float *out_rgb, float *out_T, int32_t *out_ncontrib, uint64_t *stats,
                                       uint32_t *masks, void *stream)
{
    LGS_REQUIRE(stats != nullptr && masks != nullptr, "lgs_render_debug: stats and masks are required");
    return render_batch(variant, cameras, num_views, ranges, values, splats, out_rgb, out_T, out_ncontrib, stats,
                        nullptr, nullptr, 0, masks, nullptr, 0, stream);
}

extern "C" lgs_status lgs_render(int32_t variant, const lgs_camera *camera, const uint32_t *ranges,
                                 const uint32_t *values, const float *splats, float *out_rgb, float *out_T,
                                 int32_t *out_ncontrib, uint64_t *stats, void *stream)
{
    LGS_REQUIRE(camera != nullptr, "lgs_render: invalid camera");
    return lgs_render_batch(variant, camera, 1, ranges, values, splats, out_rgb, out_T, out_ncontrib, stats, nullptr,
                            nullptr, 0, nullptr, 0, stream);
}
