// Render kernel: front-to-back alpha blending of each 16x16 tile, with the
// three Local-GS stages re-derived for 64-lane wavefronts (Sec. III).
//
// One workgroup of 256 lanes per tile; wavefront w covers the 16x4 pixel
// strip of rows 4w..4w+3 (the paper uses 16x2 strips for 32-lane warps,
// Sec. III-C-1).  Batches of up to 256 list entries are staged in LDS by the
// whole workgroup, one entry per lane.
//
// Variants (cumulative ablation ladder of the paper):
//   PLAIN       baseline loop (Alg. 1, baseline column): per-pixel quadratic
//               in screen coordinates, per-lane skip below 1/255, per-lane
//               break at T < 1e-4.
//   HOIST       + tile-local hoisting (Sec. III-B): staging computes
//               V = H(delta) [a, b, c, log2 o] once per (tile, Gaussian); each
//               lane evaluates the exponent as a 5-FMA dot product with its
//               fixed basis [x'^2, x'y', y'^2, x', y', 1].
//   HOIST_CULL  + wavefront culling (Sec. III-C): staging also evaluates the
//               tight vertical span of the footprint over the tile's columns
//               (cases A/B/C) and turns it into a 4-bit mask, one bit per
//               16x4 strip; a wavefront whose bit is 0 skips the Gaussian with
//               a scalar branch.
//   LOCAL       + uniform blending (Sec. III-D): the wavefront iterates only
//               over the set bits of a ballot of its mask bits (no per-entry
//               test at all), the blend is branch-free (alpha zeroed by a
//               select in the log2 domain, w = alpha T, C += c w, T -= w under
//               a per-lane live predicate), and termination is a wave-wide
//               ballot vote.
//
// Precision.  R = double evaluates the exponent and the transmittance in
// double (gfx950 issues FP64 FMA at the FP32 rate), so the expanded tile-local
// polynomial carries no cancellation error and every variant computes the
// same float32 exponent: the ladder differs only by rounding of T.
// R = float is the paper's single-precision arithmetic.  The exponential
// itself is v_exp_f32 of a float32 log2-domain exponent in every variant.
#include "common.hpp"

namespace lgs {
namespace {

enum Variant { kPlain = 0, kHoist = 1, kHoistCull = 2, kLocal = 3 };

struct RenderArgs {
    const uint2 *ranges;
    const uint32_t *values;
    const float2 *means2d;
    const float4 *conic_opacity;
    const float *rgb;
    float *out_rgb;
    float *out_T;
    int32_t *out_nc;
    unsigned long long *stats;
    int W, H, tiles_x, num_tiles;
    float bg0, bg1, bg2;
};

// log2(1/255) rounded to float: the alpha floor in the log2 domain
constexpr float kLog2AlphaMin = -7.99435343685885793f;
constexpr float kAlphaMinF = 1.0f / 255.0f;

// staged entry of a batch
template <typename R>
struct Hoisted {          // A, B, C, D, E, F (exponent in the log2 domain)
    R v[6];
};
struct PlainEntry {       // screen-space mean, conic, log2 opacity / opacity
    float mx, my, a, b, c, lo;
};

// workgroup index -> tile, so that each XCD (dispatch is round-robin over 8)
// processes a contiguous band of tiles and shares their splats in its L2
__device__ __forceinline__ int xcd_tile(int b, int G)
{
    const int q = G >> 3, r = G & 7, x = b & 7, k = b >> 3;
    return x * q + (x < r ? x : r) + k;
}

// Tight vertical span (Sec. III-C-2, cases A/B/C and the mirrored minimum)
// of the ellipse a x^2 + 2b x y + c y^2 <= tau over x in [x0, x1] (relative to
// the centre), mapped to a 4-bit mask of 4-row strips of the tile.
__device__ __forceinline__ uint32_t strip_mask(double a, double b, double c, double tau, double x0, double x1,
                                               double my, int ty0, int H)
{
    if (!(tau > 0.0)) return 0u;
    const double det = a * c - b * b;
    if (!(det > 0.0) || !(a > 0.0) || !(c > 0.0)) return 0xFu;
    const double dy = sqrt(a * tau / det);
    double ymax, ymin;
    // upper boundary: peak at x = -b dy / a
    if (-b * dy < a * x0) {                      // case A: peak left of the columns
        const double arg = c * tau - det * x0 * x0;
        if (arg < 0.0) return 0u;
        ymax = (-b * x0 + sqrt(arg)) / c;
    } else if (-b * dy > a * x1) {               // case B: peak right of the columns
        const double arg = c * tau - det * x1 * x1;
        if (arg < 0.0) return 0u;
        ymax = (-b * x1 + sqrt(arg)) / c;
    } else {
        ymax = dy;                                // case C
    }
    // lower boundary: trough at x = +b dy / a (signs of the linear terms reversed)
    if (b * dy < a * x0) {
        const double arg = c * tau - det * x0 * x0;
        if (arg < 0.0) return 0u;
        ymin = (-b * x0 - sqrt(arg)) / c;
    } else if (b * dy > a * x1) {
        const double arg = c * tau - det * x1 * x1;
        if (arg < 0.0) return 0u;
        ymin = (-b * x1 - sqrt(arg)) / c;
    } else {
        ymin = -dy;
    }
    const double lo = ceil(my + ymin - 1e-3), hi = floor(my + ymax + 1e-3);
    int r0 = (int)fmax(lo, (double)ty0), r1 = (int)fmin(hi, (double)(ty0 + kTile - 1));
    if (r1 > H - 1) r1 = H - 1;
    if (!(lo <= (double)(ty0 + kTile - 1)) || !(hi >= (double)ty0) || r0 > r1) return 0u;
    const int w0 = (r0 - ty0) >> 2, w1 = (r1 - ty0) >> 2;
    return ((1u << (w1 - w0 + 1)) - 1u) << w0;
}

template <int V, typename R, bool STATS>
__global__ __launch_bounds__(kBlock) void render_kernel(RenderArgs args)
{
    constexpr bool kHoisted = V != kPlain;
    constexpr bool kCull = V == kHoistCull || V == kLocal;
    using Entry = typename std::conditional<kHoisted, Hoisted<R>, PlainEntry>::type;
    __shared__ Entry s_e[kBlock];
    __shared__ float4 s_c[kBlock];
    __shared__ uint8_t s_m[kBlock];
    __shared__ int s_alive[kBlock / 64];

    const int tile = xcd_tile(blockIdx.x, args.num_tiles);
    const int tx = tile % args.tiles_x, ty = tile / args.tiles_x;
    const int lane = __lane_id(), wid = threadIdx.x >> 6;
    const int lx = lane & 15, ly = (wid << 2) | (lane >> 4);
    const int px = tx * kTile + lx, py = ty * kTile + ly;
    const bool inside = px < args.W && py < args.H;
    // tile-local frame: origin at the tile centre, so pixel coordinates are
    // the exact values -7.5 .. 7.5
    const double ox = tx * kTile + 7.5, oy = ty * kTile + 7.5;
    const R xl = (R)(lx - 7.5), yl = (R)(ly - 7.5);
    const R bxx = xl * xl, bxy = xl * yl, byy = yl * yl;
    const R gx = (R)px, gy = (R)py;

    R T = (R)1;
    float C0 = 0.f, C1 = 0.f, C2 = 0.f;
    int32_t last = 0;
    bool live = inside;
    bool wave_live = __ballot(live) != 0ull;
    unsigned long long st_seen = 0, st_eval = 0, st_staged = 0;

    const uint2 range = args.ranges[tile];
    const double tau_rel = sizeof(R) == 8 ? 1e-6 : 1e-4, tau_abs = sizeof(R) == 8 ? 1e-5 : 2e-3;

    for (uint32_t base = range.x; base < range.y; base += kBlock) {
        // workgroup-wide vote: stop fetching once every pixel has terminated
        const bool any = __ballot(live) != 0ull;
        if (lane == 0) s_alive[wid] = any;
        __syncthreads();
        if (!(s_alive[0] | s_alive[1] | s_alive[2] | s_alive[3])) break;
        const int nb = (int)min((uint32_t)kBlock, range.y - base);

        // ---- cooperative staging: one list entry per lane ----
        if ((int)threadIdx.x < nb) {
            const uint32_t g = args.values[base + threadIdx.x];
            const float2 m = args.means2d[g];
            const float4 co = args.conic_opacity[g];
            s_c[threadIdx.x] = make_float4(args.rgb[3 * g], args.rgb[3 * g + 1], args.rgb[3 * g + 2], 0.f);
            const float lo = __builtin_amdgcn_logf(co.w);   // v_log_f32 (log2)
            if constexpr (kHoisted) {
                // Eq. hoist_transform with the log2(e) scale folded in
                const R L = (R)kLog2e;
                const R a = co.x, b = co.y, c = co.z;
                const R dx = (R)((double)m.x - ox), dy = (R)((double)m.y - oy);
                Hoisted<R> h;
                h.v[0] = (R)(-0.5) * L * a;
                h.v[1] = -L * b;
                h.v[2] = (R)(-0.5) * L * c;
                h.v[3] = L * (a * dx + b * dy);
                h.v[4] = L * (b * dx + c * dy);
                h.v[5] = (R)lo - (R)0.5 * L * (a * dx * dx + (R)2 * b * dx * dy + c * dy * dy);
                s_e[threadIdx.x] = h;
                if constexpr (kCull) {
                    const double tau = 2.0 * ((double)lo - (double)kLog2AlphaMin) / kLog2e * (1.0 + tau_rel) + tau_abs;
                    const double x0 = (double)(tx * kTile) - (double)m.x;
                    s_m[threadIdx.x] = (uint8_t)strip_mask(co.x, co.y, co.z, tau, x0, x0 + (kTile - 1), (double)m.y,
                                                           ty * kTile, args.H);
                }
            } else {
                PlainEntry e;
                e.mx = m.x; e.my = m.y; e.a = co.x; e.b = co.y; e.c = co.z;
                e.lo = sizeof(R) == 8 ? lo : co.w;
                s_e[threadIdx.x] = e;
            }
        }
        if (STATS) st_staged += nb;
        __syncthreads();

        if constexpr (V == kLocal) {
            // ---- Local-GS: ballot-compacted, branch-free blend ----
            if (wave_live) {
                for (int c0 = 0; c0 < nb && wave_live; c0 += 64) {
                    const int j = c0 + lane;
                    const bool bit = j < nb && ((s_m[j] >> wid) & 1u);
                    uint64_t bits = __ballot(bit);
                    const int chunk = min(64, nb - c0);
                    int consumed = chunk;
                    while (bits) {
                        const int k = __builtin_ctzll(bits);
                        bits &= bits - 1ull;
                        const int jj = c0 + k;
                        const Hoisted<R> h = s_e[jj];
                        const float4 f = s_c[jj];
                        const R s = fma(h.v[0], bxx, fma(h.v[1], bxy, fma(h.v[2], byy,
                                    fma(h.v[3], xl, fma(h.v[4], yl, h.v[5])))));
                        const float s32 = (float)s;
                        const float al = fminf(__builtin_amdgcn_exp2f(s32), kAlphaMax);
                        const R alpha = s32 >= kLog2AlphaMin ? (R)al : (R)0;
                        const R w = alpha * T;
                        const R Tn = T - w;
                        const bool lv = live && !(Tn < (R)kTMin);
                        const float w32 = lv ? (float)w : 0.f;
                        C0 = fmaf(f.x, w32, C0);
                        C1 = fmaf(f.y, w32, C1);
                        C2 = fmaf(f.z, w32, C2);
                        T = lv ? Tn : T;
                        last = (lv && alpha > (R)0) ? (int32_t)(base + jj - range.x + 1) : last;
                        live = lv;
                        if (STATS) st_eval++;
                        if (__ballot(live) == 0ull) {
                            wave_live = false;
                            consumed = k + 1;
                            break;
                        }
                    }
                    if (STATS) st_seen += consumed;
                }
            }
        } else {
            // ---- baseline control flow (per-lane skip and break) ----
            bool done = !live;
            for (int j = 0; j < nb; ++j) {
                if (done) break;
                if (STATS) st_seen++;
                if constexpr (kCull) {
                    const uint32_t mk = __builtin_amdgcn_readfirstlane((uint32_t)s_m[j]);
                    if (!((mk >> wid) & 1u)) continue;          // uniform: whole wavefront skips
                }
                if (STATS) st_eval++;
                const float4 f = s_c[j];
                float al;
                bool keep;
                if constexpr (kHoisted) {
                    const Hoisted<R> h = s_e[j];
                    const R s = fma(h.v[0], bxx, fma(h.v[1], bxy, fma(h.v[2], byy,
                                fma(h.v[3], xl, fma(h.v[4], yl, h.v[5])))));
                    const float s32 = (float)s;
                    al = fminf(__builtin_amdgcn_exp2f(s32), kAlphaMax);
                    keep = s32 >= kLog2AlphaMin;
                } else {
                    const PlainEntry e = s_e[j];
                    if constexpr (sizeof(R) == 8) {
                        const double dx = (double)px - (double)e.mx, dy = (double)py - (double)e.my;
                        const double q = (double)e.a * dx * dx + 2.0 * (double)e.b * dx * dy + (double)e.c * dy * dy;
                        const double s = (double)e.lo - 0.5 * kLog2e * q;
                        const float s32 = (float)s;
                        al = fminf(__builtin_amdgcn_exp2f(s32), kAlphaMax);
                        keep = s32 >= kLog2AlphaMin;
                    } else {
                        // the 3DGS expression, in float
                        const float dx = e.mx - (float)gx, dy = e.my - (float)gy;
                        const float power = -0.5f * (e.a * dx * dx + e.c * dy * dy) - e.b * dx * dy;
                        al = fminf(e.lo * __builtin_amdgcn_exp2f(power * (float)kLog2e), kAlphaMax);
                        keep = al >= kAlphaMinF;
                    }
                }
                if (!keep) continue;
                const R alpha = (R)al;
                const R test = T * ((R)1 - alpha);
                if (test < (R)kTMin) { done = true; live = false; break; }
                const float w32 = (float)(alpha * T);
                C0 = fmaf(f.x, w32, C0);
                C1 = fmaf(f.y, w32, C1);
                C2 = fmaf(f.z, w32, C2);
                T = test;
                last = (int32_t)(base + j - range.x + 1);
            }
        }
    }
    if (inside) {
        const int64_t HW = (int64_t)args.W * args.H;
        const int64_t p = (int64_t)py * args.W + px;
        const float Tf = (float)T;
        args.out_rgb[p] = C0 + Tf * args.bg0;
        args.out_rgb[HW + p] = C1 + Tf * args.bg1;
        args.out_rgb[2 * HW + p] = C2 + Tf * args.bg2;
        args.out_T[p] = Tf;
        args.out_nc[p] = last;
    }
    if (STATS) {
        // a lane only ever leaves the loop, so the wavefront's step counts are
        // the per-lane maxima; lane evaluations are the per-lane sum
        unsigned long long seen = st_seen, ev = st_eval, lanes = (V == kLocal) ? st_eval * 64ull : st_eval;
        if (V != kLocal) {
            for (int off = 32; off > 0; off >>= 1) {
                seen = max(seen, (unsigned long long)__shfl_xor(seen, off, 64));
                ev = max(ev, (unsigned long long)__shfl_xor(ev, off, 64));
                lanes += __shfl_xor(lanes, off, 64);
            }
        }
        if (lane == 0) {
            atomicAdd(&args.stats[0], seen);
            atomicAdd(&args.stats[1], ev);
            atomicAdd(&args.stats[3], lanes);
        }
        if (threadIdx.x == 0) atomicAdd(&args.stats[2], st_staged);
    }
}

template <int V, typename R>
void launch_render(const RenderArgs &a, bool stats, hipStream_t s)
{
    if (stats) hipLaunchKernelGGL((render_kernel<V, R, true>), dim3(a.num_tiles), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((render_kernel<V, R, false>), dim3(a.num_tiles), dim3(kBlock), 0, s, a);
}

}  // namespace
}  // namespace lgs

using namespace lgs;

extern "C" lgs_status lgs_render(int32_t variant, const lgs_camera *camera, const uint32_t *ranges,
                                 const uint32_t *values, const float *means2d, const float *conic_opacity,
                                 const float *rgb, float *out_rgb, float *out_T, int32_t *out_ncontrib,
                                 uint64_t *stats, void *stream)
{
    Cam cam;
    LGS_REQUIRE(cam_from(camera, cam), "lgs_render: invalid camera");
    const int v = variant & 0xF;
    const bool fp32 = (variant & LGS_RENDER_FP32) != 0;
    LGS_REQUIRE(v >= 0 && v <= 3 && (variant & ~0x1F) == 0, "lgs_render: unknown variant %d", variant);
    LGS_REQUIRE(ranges && out_rgb && out_T && out_ncontrib, "lgs_render: null argument");
    LGS_REQUIRE(((uintptr_t)ranges % 8 == 0) && (means2d == nullptr || (uintptr_t)means2d % 8 == 0)
                    && (conic_opacity == nullptr || (uintptr_t)conic_opacity % 16 == 0),
                "lgs_render: misaligned ranges/means2d/conic_opacity");
    RenderArgs a;
    a.ranges = reinterpret_cast<const uint2 *>(ranges);
    a.values = values;
    a.means2d = reinterpret_cast<const float2 *>(means2d);
    a.conic_opacity = reinterpret_cast<const float4 *>(conic_opacity);
    a.rgb = rgb;
    a.out_rgb = out_rgb; a.out_T = out_T; a.out_nc = out_ncontrib;
    a.stats = reinterpret_cast<unsigned long long *>(stats);
    a.W = cam.W; a.H = cam.H; a.tiles_x = cam.tiles_x; a.num_tiles = cam.tiles_x * cam.tiles_y;
    a.bg0 = cam.bg[0]; a.bg1 = cam.bg[1]; a.bg2 = cam.bg[2];
    hipStream_t s = as_stream(stream);
    const bool st = stats != nullptr;
    if (fp32) {
        switch (v) {
        case kPlain: launch_render<kPlain, float>(a, st, s); break;
        case kHoist: launch_render<kHoist, float>(a, st, s); break;
        case kHoistCull: launch_render<kHoistCull, float>(a, st, s); break;
        default: launch_render<kLocal, float>(a, st, s); break;
        }
    } else {
        switch (v) {
        case kPlain: launch_render<kPlain, double>(a, st, s); break;
        case kHoist: launch_render<kHoist, double>(a, st, s); break;
        case kHoistCull: launch_render<kHoistCull, double>(a, st, s); break;
        default: launch_render<kLocal, double>(a, st, s); break;
        }
    }
    LGS_LAUNCHED("lgs_render");
    return LGS_OK;
}
