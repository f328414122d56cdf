// Backward of the blending stage (not part of the paper, which covers
// inference only).  For pixel p with contributors k (front to back), alpha_k,
// T_k = prod_{j<k} (1 - alpha_j) and final transmittance T_f:
//   C = sum_k c_k alpha_k T_k + T_f bg
//   dC/dc_k      = alpha_k T_k
//   dC/dalpha_k  = c_k T_k - R_k / (1 - alpha_k),  R_k = sum_{i>k} c_i alpha_i T_i + T_f bg
//   dT_f/dalpha_k = -T_f / (1 - alpha_k)
// so that, with gC = dL/dC and gT = dL/dT_f,
//   dL/dalpha_k = T_k (gC . c_k) - G_k / (1 - alpha_k),  G_k = gC . R_k + gT T_f.
// The replay walks each tile's list back to front from the largest last-
// contributor position in the workgroup, recovering T_k = T_{k+1} / (1 -
// alpha_k) from the stored final T and accumulating the scalar G_k on the way
// (G_{k-1} = G_k + (gC . c_k) alpha_k T_k).  Through
// alpha = o exp(-q/2) (unclamped): dalpha/do = alpha/o, dalpha/dq = -alpha/2,
// dq/dmean = -2 K d, dq/d(a, b, c) = (dx^2, 2 dx dy, dy^2).
//
// The LOCAL variant reuses the forward's hoisting and wavefront culling: each
// wavefront visits, in reverse, only the entries whose strip bit is set.  The
// nine per-Gaussian partial gradients are summed over the wavefront with lane
// swaps across its halves and row pairs and a DPP reduce-scatter inside the
// rows (no LDS traffic); the nine lanes holding the totals add them to the
// workgroup's LDS accumulators (no two on one address or bank), and the
// accumulators are flushed with one global atomic per nonzero (tile,
// Gaussian, component).  Per step the pixel math needs one reciprocal
// 1/(1 - alpha) (hardware estimate refined by one Newton step in double); T
// and G stay in double, the per-pixel partials are float.
#include "common.hpp"

#include "render_common.hpp"

namespace lgs {
namespace {

using namespace render;

constexpr int kNG = 9;   // mean x, y; conic a, b, c; opacity; r, g, b
// List entries staged per batch: 224 of the workgroup's 256 threads stage
// one each, so that the batch's LDS (entries, ids, strip bits, accumulators:
// 30.7 KB) lets five workgroups share a CU, and the kernel is held to 96
// registers, five wavefronts per SIMD (with 256 entries, 35 KB, four)
constexpr int kBatch = 224;

struct BwdArgs {
    RenderArgs r;          // ranges, values, attributes, out_T, out_nc (read)
    const float *grad_rgb;
    const float *grad_T;
    float *g_splats;       // packed gradient records, kGradF floats each
};

// offset in the record of each of the nine components above
__device__ __forceinline__ int grad_slot(int f)
{
    return f < 2 ? 4 + f : (f < 5 ? f - 2 : (f == 5 ? 3 : f));
}

// exact power-of-two factor applied to each accumulated component at the
// flush (the conic partials are summed without their -1/2, -1, -1/2)
__device__ __forceinline__ float grad_scale(int f)
{
    return f == 2 || f == 4 ? -0.5f : (f == 3 ? -1.0f : 1.0f);
}

template <int CTRL>
__device__ __forceinline__ float dpp_read(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

// One reduce-scatter step over the lane pairs of a DPP permutation: of the
// pair (x, y) the lane whose key bit is clear keeps x, the other keeps y, and
// each adds its partner's copy of the kept value.
template <int CTRL>
__device__ __forceinline__ float rs_step(float x, float y, bool hi)
{
    const float keep = hi ? y : x, send = hi ? x : y;
    return keep + dpp_read<CTRL>(send);
}

// Sums over lane halves and row pairs with the gfx950 lane swaps: of two
// values a and b, lanes 0..31 end with a summed over lanes l and l + 32 and
// lanes 32..63 with b summed likewise (32-lane swap); or rows 0 and 2 end with
// a summed over rows (0, 1), resp. (2, 3), and rows 1 and 3 with b (16-lane
// swap of the odd rows of the first operand with the even rows of the second).
__device__ __forceinline__ float halves_pair(float a, float b)
{
    const auto s = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(s[0]) + __uint_as_float(s[1]);
}

__device__ __forceinline__ float rows_pair(float a, float b)
{
    const auto s = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(s[0]) + __uint_as_float(s[1]);
}

// Sums of nine values over all 64 lanes (all lanes active), scattered: lane l
// in row r = l >> 4 at position p = l & 15 ends with the total of component
// wave_comp(l).  Components pair up over the two halves (0|1, 2|3, 4|5, 6|7),
// then over the row pairs, so that row r holds one of 0, 2, 1, 3 and one of
// 4, 6, 5, 7 (and every row component 8) summed over the four rows; inside
// the rows a DPP reduce-scatter over the row mirror (key bit 3 of p) and the
// half-row mirror (bit 2) and butterflies over the quads finish them: 25
// instructions.
__device__ __forceinline__ float wave_sums9(const float *g)
{
    const float s01 = halves_pair(g[0], g[1]), s23 = halves_pair(g[2], g[3]);
    const float s45 = halves_pair(g[4], g[5]), s67 = halves_pair(g[6], g[7]);
    float t8 = halves_pair(g[8], g[8]);
    const float q0 = rows_pair(s01, s23), q1 = rows_pair(s45, s67);
    t8 = rows_pair(t8, t8);
    const int p = __lane_id() & 15;
    const float u = rs_step<0x140>(q0, q1, (p & 8) != 0);                  // row_mirror
    t8 += dpp_read<0x140>(t8);
    float v = rs_step<0x141>(u, t8, (p & 4) != 0);                        // row_half_mirror
    v += dpp_read<0x4E>(v);                                                 // quad_perm [2,3,0,1]
    v += dpp_read<0xB1>(v);                                                 // quad_perm [1,0,3,2]
    return v;
}

// the component whose total wave_sums9 leaves in lane l; lanes 0 and 8 of
// every row and lane 4 of row 0 hold the nine totals once each
__device__ __forceinline__ int wave_comp(int l)
{
    const int r = l >> 4, p = l & 15;
    const int c = ((r & 1) << 1) | (r >> 1);       // rows hold 0, 2, 1, 3
    return p < 4 ? c : (p >= 8 && p < 12 ? 4 + c : 8);
}

__device__ __forceinline__ bool wave_owner(int l)
{
    return (l & 7) == 0 || l == 4;
}

// 1 / x for normal positive x (here 1 - alpha in [0.01, 1]): hardware
// estimate (measured relative error 2^-24.4 on that interval) and one Newton
// step, which squares it (measured 2^-48.7, a few ulps; exact for x = 1, so a
// lane that skips a Gaussian keeps its T bit for bit)
__device__ __forceinline__ double recip(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    const double e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// R is the precision of the forward's exponent (double, or float for the
// single-precision variants): the replay evaluates alpha with the same
// expression as the forward kernel it follows, so that it takes the same skip
// and clamp decisions.
//
// Grid mode: one workgroup per tile (in the order of `order`, else XCD-banded).
// Persistent mode (queue != null): blocks_per_cu workgroups per CU pop tiles
// from eight per-XCD counters (workgroup b draws from counter b % 8, which
// hands out queue positions b % 8, b % 8 + 8, ...; position -> tile through
// `order`) until the positions run out; every workgroup reaches that exit.
//
// STATS counts, per wavefront: [0] (wavefront, Gaussian) steps whose strip
// bit is set within the wavefront's replay range, [1] steps some lane takes
// (replayed), [2] (lane, Gaussian) pairs taken, [3] lane evaluations (64 per
// replayed step).
struct BwdStats {
    unsigned long long cand = 0, proc = 0, taken = 0;
};

// one staged list entry in LDS: every field a replay step reads, at fixed
// offsets from one wave-uniform base address
template <typename R>
struct alignas(16) BwdEntry {
    Hoisted<R> v;          // hoisted exponent coefficients (plain: v[5] = log2 o)
    float4 co;             // a, b, c, o
    float4 c;              // colour, 1/o
    float2 mu;             // mean
};

template <bool LOCAL, bool Q8, typename R, bool STATS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(5, 5))) void render_bwd_kernel(BwdArgs ba)
{
    __shared__ BwdEntry<R> s_e[kBatch];
    __shared__ uint32_t s_id[kBatch];
    __shared__ uint8_t s_m[kBatch];
    __shared__ float s_g[kNG][kBatch + 1];  // padded: the nine components of an entry in distinct banks
    __shared__ int s_max[kBlock / 64];
    __shared__ uint32_t s_pos;

    const RenderArgs &a = ba.r;
    BwdStats st;

    auto replay_tile = [&](const int tile) {
    const TileCtx<R> tc(a, tile, threadIdx.x >> 6, Q8);
    const int lane = __lane_id(), wid = tc.wid;
    const int px = tc.px, py = tc.py;
    const bool inside = tc.inside;
    const int tx = tc.tx, ty = tc.ty;
    const int64_t HW = (int64_t)tc.W * tc.H;
    const int64_t p = tc.pix0 + (int64_t)py * tc.W + px;           // packed pixel index
    const int64_t pc = 3 * tc.pix0 + (int64_t)py * tc.W + px;      // channel-0 index of this view
    const int last = inside ? a.out_nc[p] : 0;
    const double Tf = inside ? (double)a.out_T[p] : 1.0;
    double T = Tf;
    const float gc0 = inside ? ba.grad_rgb[pc] : 0.f, gc1 = inside ? ba.grad_rgb[HW + pc] : 0.f,
                gc2 = inside ? ba.grad_rgb[2 * HW + pc] : 0.f;
    const double gt = (inside && ba.grad_T) ? (double)ba.grad_T[p] : 0.0;
    const float *bg = a.vt.bg[tc.view];
    // G = sum_c dL/dC_c R_c + dL/dT_f T_f, R_c the colour behind the current
    // Gaussian (initially the background seen through T_f): the only
    // combination of the running colour sums that dL/dalpha needs
    double G = Tf * ((double)gc0 * bg[0] + (double)gc1 * bg[1] + (double)gc2 * bg[2] + gt);

    int wmax = last;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) wmax = max(wmax, __shfl_xor(wmax, off, 64));
    if (lane == 0) s_max[wid] = wmax;
    __syncthreads();
    const int bmax = max(max(s_max[0], s_max[1]), max(s_max[2], s_max[3]));
    const uint2 range = a.ranges[tc.tile];
    const uint32_t end = range.x + (uint32_t)bmax;

    // Two-deep software pipeline over the batches (back to front, kBatch
    // entries each): while batch i is replayed, thread t holds the attributes
    // of entry t of batch i + 1 and the Gaussian id of entry t of batch i + 2
    // in registers, so the dependent gathers overlap the replay.
    auto batch_start = [&](int64_t be) { return (uint32_t)max((int64_t)range.x, be - kBatch); };
    auto fetch_id = [&](int64_t be) -> uint32_t {
        const uint32_t bs = batch_start(be);
        return (be > (int64_t)range.x && (int64_t)threadIdx.x < be - (int64_t)bs) ? a.values[bs + threadIdx.x] : 0u;
    };
    struct Attr {
        float2 m;
        float4 co;
        float r, gg, b;
    };
    auto fetch_attr = [&](int64_t be, uint32_t g) -> Attr {
        Attr at{make_float2(0.f, 0.f), make_float4(0.f, 0.f, 0.f, 1.f), 0.f, 0.f, 0.f};
        if (be > (int64_t)range.x && (int64_t)threadIdx.x < be - (int64_t)batch_start(be)) {
            const float4 *rec = splat_rec(a.splats, g);
            at.co = rec[0];
            const float4 mr = rec[1];
            at.m = make_float2(mr.x, mr.y);
            at.r = mr.z; at.gg = mr.w; at.b = reinterpret_cast<const float *>(rec + 2)[0];
        }
        return at;
    };
    uint32_t id_cur = fetch_id(end);
    Attr at_cur = fetch_attr(end, id_cur);
    uint32_t id_next = fetch_id((int64_t)end - kBatch);

    for (int64_t bend = end; bend > (int64_t)range.x; bend -= kBatch) {
        const uint32_t bstart = (uint32_t)max((int64_t)range.x, bend - kBatch);
        const int nb = (int)(bend - bstart);
        __syncthreads();                                   // previous batch fully flushed
        if ((int)threadIdx.x < nb) {
            const int k = threadIdx.x;
            const uint32_t g = id_cur;
            const float2 m = at_cur.m;
            const float4 co = at_cur.co;
            s_id[k] = g;
            s_e[k].mu = m;
            s_e[k].co = co;
            s_e[k].c = make_float4(at_cur.r, at_cur.gg, at_cur.b, __builtin_amdgcn_rcpf(co.w));
            const float lo = __builtin_amdgcn_logf(co.w);
            if (LOCAL) {
                s_e[k].v = hoist<R>(m, co, lo, tc.ox, tc.oy);
                // strip bits of the four wavefronts (the forward's test; the
                // strips share their columns, so the ellipse's vertical span
                // over them is computed once)
                uint32_t mk = 0;
                float ymin, ymax;
                if (a.used != nullptr) {
                    mk = 0xF;                       // the forward's used-entry masks decide below
                } else if constexpr (Q8) {
                    // quadrant w: columns half (w & 1), rows half (w >> 1)
                    for (int hx = 0; hx < 2; ++hx) {
                        const float x0 = (float)(tx * kTile + 8 * hx) - m.x, x1 = x0 + 7.0f;
                        if (!column_span(co.x, co.y, co.z, lo, x0, x1, ymin, ymax)) continue;
                        for (int hy = 0; hy < 2; ++hy) {
                            const int r0 = ty * kTile + 8 * hy;
                            if (r0 > tc.H - 1) break;
                            const int r1 = min(r0 + 7, tc.H - 1);
                            if (span_meets(ymin, ymax, (float)r0 - m.y, (float)r1 - m.y)) mk |= 1u << (2 * hy + hx);
                        }
                    }
                } else {
                    const float x0 = (float)(tx * kTile) - m.x, x1 = (float)(tx * kTile + kTile - 1) - m.x;
                    if (column_span(co.x, co.y, co.z, lo, x0, x1, ymin, ymax)) {
                        for (int w = 0; w < 4; ++w) {
                            const int r0 = ty * kTile + 4 * w;
                            if (r0 > tc.H - 1) break;
                            const int r1 = min(r0 + 3, tc.H - 1);
                            if (span_meets(ymin, ymax, (float)r0 - m.y, (float)r1 - m.y)) mk |= 1u << w;
                        }
                    }
                }
                s_m[k] = (uint8_t)mk;
            } else {
                s_e[k].v.v[5] = (R)lo;
                s_m[k] = 0xF;
            }
#pragma unroll
            for (int f = 0; f < kNG; ++f) s_g[f][k] = 0.f;
        }
        __syncthreads();
        // the next batches' loads, in flight during this one's replay
        id_cur = id_next;
        at_cur = fetch_attr(bend - kBatch, id_cur);
        id_next = fetch_id(bend - 2 * (int64_t)kBatch);

        // wavefront's own range: skip entries past its last contributor
        const int wlimit = __builtin_amdgcn_readfirstlane(
            (int)min((int64_t)nb, (int64_t)range.x + wmax - (int64_t)bstart));
        for (int c0 = ((wlimit - 1) >> 6) << 6; wlimit > 0 && c0 >= 0; c0 -= 64) {
            const int j = c0 + lane;
            // candidates: the entries some pixel of this sub-tile blended in
            // the forward (its used-entry masks; an entry outside them has
            // alpha < 1/255 or comes after termination at every pixel), else
            // the entries the tight-box test keeps
            bool bit = j < wlimit;
            if (a.used != nullptr) {
                const uint32_t p = bstart + (uint32_t)j;
                const int64_t wd = used_word(range.x, tc.tile, p);
                bit = bit && (wd >= a.used_plane
                              || ((a.used[(int64_t)wid * a.used_plane + wd] >> ((p - range.x) & 63u)) & 1ull));
            } else {
                bit = bit && ((s_m[j] >> wid) & 1u);
            }
            uint64_t bits = __ballot(bit);
            if (STATS) st.cand += (unsigned long long)__popcll(bits);
            while (bits) {
                const int kk = 63 - __builtin_clzll(bits);
                bits &= ~(1ull << kk);
                const int k = __builtin_amdgcn_readfirstlane(c0 + kk);   // uniform: scalar addressing
                const BwdEntry<R> &e = s_e[k];
                const int pos1 = (int)(bstart + k - range.x) + 1;
                const float4 co = e.co;
                const float2 m = e.mu;
                // raw: the unclamped alpha o exp(-q/2), as the forward computed it
                float raw;
                bool keep;
                if (LOCAL) {
                    const float s32 = (float)dot_exponent(e.v, tc);
                    raw = __builtin_amdgcn_exp2f(s32);
                    keep = s32 >= kLog2AlphaMin;
                } else if constexpr (sizeof(R) == 8) {
                    const double dxd = (double)px - (double)m.x, dyd = (double)py - (double)m.y;
                    const double q = (double)co.x * dxd * dxd + 2.0 * (double)co.y * dxd * dyd
                                     + (double)co.z * dyd * dyd;
                    const float s32 = (float)((double)e.v.v[5] - 0.5 * kLog2e * q);
                    raw = __builtin_amdgcn_exp2f(s32);
                    keep = s32 >= kLog2AlphaMin;
                } else {
                    // the plain single-precision forward: o * exp(power) in float
                    const float ex = m.x - (float)px, ey = m.y - (float)py;
                    const float power = -0.5f * (co.x * ex * ex + co.z * ey * ey) - co.y * ex * ey;
                    raw = co.w * __builtin_amdgcn_exp2f(power * (float)kLog2e);
                    keep = fminf(raw, kAlphaMax) >= kAlphaMinF;
                }
                const float dx = (float)px - m.x, dy = (float)py - m.y;
                const bool act = pos1 <= last && keep;
                if (__ballot(act) == 0ull) continue;          // no lane of the wavefront takes this Gaussian
                if (STATS) { st.proc++; st.taken += act ? 1ull : 0ull; }
                // Branch-free from here: a lane that does not take the Gaussian
                // uses alpha = 0, so T (times 1/(1 - 0) = 1) and R are unchanged
                // and every partial is zero.
                const bool under = raw < kAlphaMax;              // not clamped
                // min(raw, 0.99) for raw >= 0 (as a median: no canonicalising)
                const float alf = act ? __builtin_amdgcn_fmed3f(raw, 0.f, kAlphaMax) : 0.f;
                const double al = (double)alf;
                const double inv = recip(1.0 - al);
                T = T * inv;                                     // T before this Gaussian
                const double w = al * T;
                const float4 f = e.c;
                // dL/dalpha = T sum_c dL/dC_c c_c - G / (1 - alpha); then the
                // Gaussian's own weighted colour joins G
                const double gcc = (double)fmaf(gc2, f.z, fmaf(gc1, f.y, gc0 * f.x));
                const double dLda = fma(T, gcc, -G * inv);
                G = fma(gcc, w, G);
                // the per-pixel partials are single terms (no long sums):
                // float is enough for them; no gradient through the clamp
                float g[kNG];
                const float wf = (float)w;
                g[6] = gc0 * wf; g[7] = gc1 * wf; g[8] = gc2 * wf;
                const float dLdaf = (act && under) ? (float)dLda : 0.f;
                // A = alpha dL/dalpha = -2 dL/dq; the conic partials are
                // accumulated as A (dx^2, dx dy, dy^2) and scaled by
                // (-1/2, -1, -1/2) once per entry in the flush
                const float A = alf * dLdaf;
                const float Ax = A * dx, Ay = A * dy;
                g[0] = fmaf(co.x, Ax, co.y * Ay);
                g[1] = fmaf(co.y, Ax, co.z * Ay);
                g[2] = Ax * dx;
                g[3] = Ax * dy;
                g[4] = Ay * dy;
                g[5] = dLdaf * raw * f.w;                       // dalpha/do = raw / o
                {
                    static_assert(kNG == 9, "wave_sums9 handles nine components");
                    const float tot = wave_sums9(g);
                    // (a zero total adds nothing; testing for it cost more than the add)
                    if (wave_owner(lane)) atomicAdd(&s_g[wave_comp(lane)][k], tot);
                }
            }
        }
        __syncthreads();
        // one global atomic per nonzero (tile, Gaussian, component), work
        // item t = 9 * entry + component: the 64 lanes of an atomic
        // instruction cover the records of about seven entries rather than
        // one component of 64 records
        for (int t = threadIdx.x; t < nb * kNG; t += kBlock) {
            const int k = t / kNG, f = t - k * kNG;
            const float v = s_g[f][k] * grad_scale(f);
            if (v != 0.f) unsafeAtomicAdd(ba.g_splats + (uint64_t)s_id[k] * kGradF + grad_slot(f), v);
        }
    }
    };  // replay_tile

    // one call site of the tile body for both modes (two would be inlined
    // twice and the register allocation would take the larger of both)
    const uint32_t x = blockIdx.x & (kQueues - 1);
    for (int round = 0;; ++round) {
        int tile;
        if (a.queue == nullptr) {
            if (round > 0) break;
            tile = a.order ? (int)a.order[blockIdx.x] : xcd_tile(blockIdx.x, a.num_tiles);
        } else {
            __syncthreads();                                // s_pos of the last round read by all
            if (threadIdx.x == 0) s_pos = atomicAdd(a.queue + x * kQueueStride, 1u);
            __syncthreads();
            const uint64_t pos = (uint64_t)s_pos * kQueues + x;
            if (pos >= (uint64_t)a.num_tiles) break;
            tile = a.order ? (int)a.order[pos] : (int)pos;
        }
        replay_tile(tile);
    }
    if (STATS) {
        unsigned long long cand = st.cand, proc = st.proc, taken = st.taken;
        for (int off = 32; off > 0; off >>= 1) taken += (unsigned long long)__shfl_xor(taken, off, 64);
        if (__lane_id() == 0) {
            atomicAdd(&a.stats[0], cand);
            atomicAdd(&a.stats[1], proc);
            atomicAdd(&a.stats[2], taken);
            atomicAdd(&a.stats[3], 64ull * proc);
        }
    }
}

template <bool LOCAL, bool Q8, typename R>
void launch_bwd(bool stats, dim3 g, hipStream_t s, const BwdArgs &a)
{
    if (stats) hipLaunchKernelGGL((render_bwd_kernel<LOCAL, Q8, R, true>), g, dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((render_bwd_kernel<LOCAL, Q8, R, false>), g, dim3(kBlock), 0, s, a);
}

}  // namespace
}  // namespace lgs

using namespace lgs;

extern "C" lgs_status lgs_render_backward_batch(int32_t variant, const lgs_camera *cameras, int32_t num_views,
                                                int64_t n_elem, const uint32_t *ranges, const uint32_t *values,
                                                const float *splats, const float *out_T,
                                                const int32_t *out_ncontrib, const float *grad_rgb,
                                                const float *grad_T, float *g_splats, const uint32_t *tile_order,
                                                uint32_t *queue, int32_t blocks_per_cu, uint64_t *stats,
                                                const uint64_t *used_masks, int64_t used_mask_words, void *stream)
{
    LGS_REQUIRE(num_views >= 1 && num_views <= kMaxViews, "lgs_render_backward: num_views must be 1..%d", kMaxViews);
    LGS_REQUIRE(cameras != nullptr, "lgs_render_backward: invalid camera");
    Cam cams[kMaxViews];
    for (int v = 0; v < num_views; ++v)
        LGS_REQUIRE(cam_from(&cameras[v], cams[v]), "lgs_render_backward: invalid camera %d", v);
    const int v = variant & 0xF;
    LGS_REQUIRE(v == LGS_RENDER_PLAIN || v == LGS_RENDER_LOCAL, "lgs_render_backward: variant must be PLAIN or LOCAL");
    const bool fp32 = (variant & LGS_RENDER_FP32) != 0;
    const bool q8 = (variant & LGS_RENDER_Q8) != 0;
    LGS_REQUIRE(n_elem >= 0, "lgs_render_backward: n < 0");
    LGS_REQUIRE(ranges && out_T && out_ncontrib && grad_rgb, "lgs_render_backward: null input");
    LGS_REQUIRE(n_elem == 0 || (values && splats && g_splats), "lgs_render_backward: null argument");
    LGS_REQUIRE(((uintptr_t)ranges % 8 == 0) && ((uintptr_t)splats % 16 == 0) && ((uintptr_t)g_splats % 4 == 0),
                "lgs_render_backward: ranges must be 8-byte, splats 16-byte and g_splats 4-byte aligned");
    LGS_REQUIRE(used_masks == nullptr
                    || (v == LGS_RENDER_LOCAL && used_mask_words >= 4 && (uintptr_t)used_masks % 8 == 0),
                "lgs_render_backward: used_masks need the LOCAL variant, 8-byte alignment and at least 4 words");
    hipStream_t s = as_stream(stream);
    if (!(variant & LGS_BWD_ACCUMULATE)) fill_async<float>(g_splats, 0.f, n_elem * kGradF, s);
    BwdArgs a;
    a.r = render::make_args(cams, num_views, ranges, values, splats, nullptr, const_cast<float *>(out_T),
                            const_cast<int32_t *>(out_ncontrib), stats);
    a.r.order = tile_order;
    a.r.global_origin = (variant & LGS_RENDER_GLOBAL) != 0;
    a.r.used = const_cast<uint64_t *>(used_masks);
    a.r.used_plane = used_masks ? used_mask_words / 4 : 0;
    a.grad_rgb = grad_rgb; a.grad_T = grad_T;
    a.g_splats = g_splats;
    if (a.r.num_tiles > 0) {
        dim3 g(a.r.num_tiles);
        if (queue != nullptr) {
            static_assert(kQueues * kQueueStride == LGS_QUEUE_WORDS, "queue block size");
            fill_async<uint32_t>(queue, 0u, kQueues * kQueueStride, s);
            a.r.queue = queue;
            const int per = blocks_per_cu > 0 ? blocks_per_cu : 4;
            g = dim3((unsigned)((device_cus() * per + kQueues - 1) / kQueues * kQueues));
        }
        const bool st = stats != nullptr;
        if (fp32) {
            if (v == LGS_RENDER_PLAIN) launch_bwd<false, false, float>(st, g, s, a);
            else if (q8) launch_bwd<true, true, float>(st, g, s, a);
            else launch_bwd<true, false, float>(st, g, s, a);
        } else {
            if (v == LGS_RENDER_PLAIN) launch_bwd<false, false, double>(st, g, s, a);
            else if (q8) launch_bwd<true, true, double>(st, g, s, a);
            else launch_bwd<true, false, double>(st, g, s, a);
        }
    }
    LGS_LAUNCHED("lgs_render_backward");
    return LGS_OK;
}

extern "C" lgs_status lgs_render_backward(int32_t variant, const lgs_camera *camera, int64_t n, const uint32_t *ranges,
                                          const uint32_t *values, const float *splats, const float *out_T,
                                          const int32_t *out_ncontrib, const float *grad_rgb, const float *grad_T,
                                          float *g_splats, void *stream)
{
    return lgs_render_backward_batch(variant, camera, 1, n, ranges, values, splats, out_T, out_ncontrib, grad_rgb,
                                     grad_T, g_splats, nullptr, nullptr, 0, nullptr, nullptr, 0, stream);
}
