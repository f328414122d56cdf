// Pieces shared by the forward and backward render kernels: tile geometry,
// the hoist transform, the tight-box strip test and output helpers.
#pragma once

#include "common.hpp"

namespace lgs {
namespace render {

// log2(1/255) rounded to float: the alpha floor in the log2 domain
constexpr float kLog2AlphaMin = -7.99435343685885793f;
constexpr float kAlphaMinF = 1.0f / 255.0f;
constexpr float kLn2f = 0.693147180559945309f;

// Up to kMaxViews cameras of different sizes share one flattened tile space:
// view v owns global tiles [tile_off[v], tile_off[v+1]) and its outputs start
// at pixel pix_off[v] of the packed output buffers.

struct ViewTable {
    int V;
    int tile_off[kMaxViews + 1];
    int tiles_x[kMaxViews];
    int W[kMaxViews], H[kMaxViews];
    int64_t pix_off[kMaxViews];
    float bg[kMaxViews][3];
};

// persistent mode: one work counter per XCD, each on its own 128-byte line
constexpr int kQueues = 8;
constexpr int kQueueStride = 32;                 // uint32 words between counters

struct RenderArgs {
    const uint2 *ranges;
    const uint32_t *values;
    const float *splats;        // projected splat records
    float *out_rgb;
    float *out_T;
    int32_t *out_nc;
    unsigned long long *stats;
    uint32_t *queue;            // persistent mode: kQueues counters (zeroed before launch), else null
    const uint32_t *order;      // tile of each queue position (persistent render) or workgroup (backward), or null
    int num_tiles;              // all views
    int global_origin;          // hoisted basis at the image origin instead of the tile centre
    uint32_t *masks;            // statistics instantiation only: per-entry culling record, or null
    uint64_t *used;             // per (sub-tile, chunk) masks of the entries some pixel blended, or null
    int64_t used_plane;         // words per sub-tile plane of `used`
    ViewTable vt;
};

// Word of the used-entry masks for list position p of a tile whose list
// starts at position a (tile index t): chunks of 64 positions from a, offset
// by a >> 6 and the tile index so that no two tiles' chunks share a word
// (a plane holds capacity / 64 + tiles + 1 words).
__device__ __forceinline__ int64_t used_word(uint32_t a, int t, uint32_t p)
{
    return (int64_t)(a >> 6) + t + (int64_t)((p - a) >> 6);
}

inline void fill_views(ViewTable &vt, const Cam *cams, int V)
{
    vt.V = V;
    int t = 0;
    int64_t px = 0;
    for (int v = 0; v < V; ++v) {
        vt.tile_off[v] = t;
        vt.tiles_x[v] = cams[v].tiles_x;
        vt.W[v] = cams[v].W;
        vt.H[v] = cams[v].H;
        vt.pix_off[v] = px;
        for (int c = 0; c < 3; ++c) vt.bg[v][c] = cams[v].bg[c];
        t += cams[v].tiles_x * cams[v].tiles_y;
        px += (int64_t)cams[v].W * cams[v].H;
    }
    vt.tile_off[V] = t;
    for (int v = V; v < kMaxViews; ++v) {
        vt.tiles_x[v] = 1; vt.W[v] = 0; vt.H[v] = 0; vt.pix_off[v] = px;
        vt.bg[v][0] = vt.bg[v][1] = vt.bg[v][2] = 0.f;
    }
}

inline RenderArgs make_args(const Cam *cams, int V, const uint32_t *ranges, const uint32_t *values,
                            const float *splats, float *out_rgb, float *out_T, int32_t *out_nc, uint64_t *stats)
{
    RenderArgs a;
    a.ranges = reinterpret_cast<const uint2 *>(ranges);
    a.values = values;
    a.splats = splats;
    a.out_rgb = out_rgb; a.out_T = out_T; a.out_nc = out_nc;
    a.stats = reinterpret_cast<unsigned long long *>(stats);
    a.queue = nullptr;
    a.order = nullptr;
    a.global_origin = 0;
    a.masks = nullptr;
    a.used = nullptr;
    a.used_plane = 0;
    fill_views(a.vt, cams, V);
    a.num_tiles = a.vt.tile_off[V];
    return a;
}

// workgroup index -> tile, so that each XCD (dispatch is round-robin over 8)
// processes a contiguous band of tiles and shares their splats in its L2
__device__ __forceinline__ int xcd_tile(int b, int G)
{
    const int q = G >> 3, r = G & 7, x = b & 7, k = b >> 3;
    return x * q + (x < r ? x : r) + k;
}

// Geometry of one lane for global tile `tile` and wavefront sub-tile
// `strip` (0..3): view, pixel, output offset and the tile-local basis.  The
// sub-tiles are 16x4 row strips, or with q8 the four 8x8 quadrants.  The
// tile-local origin is the tile centre, so the basis coordinates are the
// exact values -7.5 .. 7.5 (with global_origin: the image origin, basis
// coordinates the pixel's own, as in the paper's global-coordinate
// precision baseline).  [sx0, sx1] x [sy0, sy1] is the sub-tile clipped to
// the image (empty when no pixel of it is inside).
template <typename R>
struct TileCtx {
    int tile, view, tx, ty, wid, px, py, W, H;
    int sx0, sx1, sy0, sy1;
    bool inside;
    int64_t pix0;       // first pixel of this view in the packed outputs
    double ox, oy;
    R xl, yl, bxx, bxy, byy;
    __device__ __forceinline__ TileCtx(const RenderArgs &a, int gtile, int strip, bool q8 = false)
    {
        tile = gtile;
        int v = 0;
        while (v + 1 < a.vt.V && gtile >= a.vt.tile_off[v + 1]) ++v;
        view = v;
        const int lt = gtile - a.vt.tile_off[v];
        tx = lt % a.vt.tiles_x[v];
        ty = lt / a.vt.tiles_x[v];
        W = a.vt.W[v];
        H = a.vt.H[v];
        pix0 = a.vt.pix_off[v];
        const int lane = __lane_id();
        wid = strip;
        int lx, ly;
        if (q8) {
            lx = ((wid & 1) << 3) | (lane & 7);
            ly = ((wid >> 1) << 3) | (lane >> 3);
            sx0 = tx * kTile + ((wid & 1) << 3);
            sy0 = ty * kTile + ((wid >> 1) << 3);
            sx1 = min(sx0 + 7, W - 1);
            sy1 = min(sy0 + 7, H - 1);
        } else {
            lx = lane & 15;
            ly = (wid << 2) | (lane >> 4);
            sx0 = tx * kTile;
            sy0 = ty * kTile + (wid << 2);
            sx1 = min(sx0 + kTile - 1, W - 1);
            sy1 = min(sy0 + 3, H - 1);
        }
        px = tx * kTile + lx;
        py = ty * kTile + ly;
        inside = px < W && py < H;
        if (a.global_origin) {
            ox = 0.0;
            oy = 0.0;
            xl = (R)px;
            yl = (R)py;
        } else {
            ox = tx * kTile + 7.5;
            oy = ty * kTile + 7.5;
            xl = (R)(lx - 7.5);
            yl = (R)(ly - 7.5);
        }
        bxx = xl * xl; bxy = xl * yl; byy = yl * yl;
    }
};

// Hoisted exponent coefficients (Eq. hoist_transform, log2(e) folded in):
// log2 alpha = A x'^2 + B x'y' + C y'^2 + D x' + E y' + F
template <typename R>
struct Hoisted {
    R v[6];
};

template <typename R>
__device__ __forceinline__ Hoisted<R> hoist(float2 m, float4 co, float lo, double ox, double oy)
{
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
    return h;
}

// the per-lane 5-FMA dot product with [x'^2, x'y', y'^2, x', y', 1]
template <typename R>
__device__ __forceinline__ R dot_exponent(const Hoisted<R> &h, const TileCtx<R> &tc)
{
    return fma(h.v[0], tc.bxx, fma(h.v[1], tc.bxy, fma(h.v[2], tc.byy, fma(h.v[3], tc.xl, fma(h.v[4], tc.yl, h.v[5])))));
}

// Does the footprint alpha >= 1/255, i.e. q <= tau with
// tau = 2 ln 2 (log2 o - log2(1/255)), meet the rectangle [x0, x1] x [y0, y1]
// (coordinates relative to the splat centre)?  Tight vertical span of the
// ellipse over [x0, x1] (Sec. III-C-2: cases A/B/C for the top, the mirrored
// cases for the bottom), then an interval test against [y0, y1].
// Evaluated in float on a slightly larger ellipse, tau' = tau (1 + 1e-3) +
// 1e-2: the enlargement exceeds every float rounding error of the test (the
// product b^2 is split exactly so det keeps full relative accuracy, the
// square-root arguments stay >= c (tau' - tau) at the true tangent points,
// and the hardware reciprocal and square root used for the quotients are
// within 1 ulp), so a Gaussian that can reach alpha >= 1/255 at a pixel of
// the strip is never culled.
// Vertical extent [ymin, ymax] of that enlarged ellipse over the columns
// [x0, x1]; false when it misses the columns entirely.  A degenerate conic
// (not positive definite) gives the whole line.
__device__ __forceinline__ bool column_span(float a, float b, float c, float lo, float x0, float x1, float &ymin,
                                            float &ymax)
{
    float tau = 2.0f * kLn2f * (lo - kLog2AlphaMin);
    if (!(tau > 0.0f)) return false;
    tau = fmaf(tau, 1e-3f, tau) + 1e-2f;
    const float p = b * b;
    const float pe = fmaf(b, b, -p);
    const float det = fmaf(a, c, -p) - pe;
    if (!(det > 0.0f) || !(a > 0.0f) || !(c > 0.0f)) {
        ymin = -INFINITY;
        ymax = INFINITY;
        return true;
    }
    const float rc = __builtin_amdgcn_rcpf(c);
    const float dy = __builtin_amdgcn_sqrtf(a * tau * __builtin_amdgcn_rcpf(det));
    const float bdy = b * dy;
    if (-bdy < a * x0) {                       // case A: peak left of the columns
        const float arg = c * tau - det * x0 * x0;
        if (arg < 0.0f) return false;
        ymax = (-b * x0 + __builtin_amdgcn_sqrtf(arg)) * rc;
    } else if (-bdy > a * x1) {                // case B: peak right of the columns
        const float arg = c * tau - det * x1 * x1;
        if (arg < 0.0f) return false;
        ymax = (-b * x1 + __builtin_amdgcn_sqrtf(arg)) * rc;
    } else {
        ymax = dy;                             // case C: peak inside
    }
    if (bdy < a * x0) {                        // mirrored cases for the bottom
        const float arg = c * tau - det * x0 * x0;
        if (arg < 0.0f) return false;
        ymin = (-b * x0 - __builtin_amdgcn_sqrtf(arg)) * rc;
    } else if (bdy > a * x1) {
        const float arg = c * tau - det * x1 * x1;
        if (arg < 0.0f) return false;
        ymin = (-b * x1 - __builtin_amdgcn_sqrtf(arg)) * rc;
    } else {
        ymin = -dy;
    }
    return true;
}

// does the span meet the rows [y0, y1]?
__device__ __forceinline__ bool span_meets(float ymin, float ymax, float y0, float y1)
{
    return ymax >= y0 - 1e-3f && ymin <= y1 + 1e-3f;
}

// the whole test for one rectangle
__device__ __forceinline__ bool strip_hit(float a, float b, float c, float lo, float x0, float x1, float y0,
                                          float y1)
{
    float ymin, ymax;
    return column_span(a, b, c, lo, x0, x1, ymin, ymax) && span_meets(ymin, ymax, y0, y1);
}

template <typename R>
__device__ __forceinline__ void write_pixel(const RenderArgs &a, const TileCtx<R> &tc, float C0, float C1, float C2,
                                            float T, int32_t last)
{
    if (!tc.inside) return;
    const int64_t HW = (int64_t)tc.W * tc.H;
    const int64_t p = (int64_t)tc.py * tc.W + tc.px;
    float *rgb = a.out_rgb + 3 * tc.pix0;
    const float *bg = a.vt.bg[tc.view];
    rgb[p] = C0 + T * bg[0];
    rgb[HW + p] = C1 + T * bg[1];
    rgb[2 * HW + p] = C2 + T * bg[2];
    a.out_T[tc.pix0 + p] = T;
    a.out_nc[tc.pix0 + p] = last;
}

// Counters: [0] (wavefront, Gaussian) steps met by live wavefronts, [1] steps
// evaluated, [2] entries staged, [3] lane evaluations (64 per evaluated step).
// Per-lane counts are reduced to the wavefront maximum (a lane only ever
// leaves the loop, so the last lane to leave saw every step).
template <bool PER_WAVE_STAGED>
__device__ __forceinline__ void flush_stats(const RenderArgs &a, unsigned long long seen, unsigned long long ev,
                                            unsigned long long staged)
{
    for (int off = 32; off > 0; off >>= 1) {
        seen = max(seen, (unsigned long long)__shfl_xor(seen, off, 64));
        ev = max(ev, (unsigned long long)__shfl_xor(ev, off, 64));
    }
    if (__lane_id() == 0) {
        atomicAdd(&a.stats[0], seen);
        atomicAdd(&a.stats[1], ev);
        atomicAdd(&a.stats[3], ev * 64ull);
        if (PER_WAVE_STAGED) atomicAdd(&a.stats[2], staged);
    }
    if (!PER_WAVE_STAGED && threadIdx.x == 0) atomicAdd(&a.stats[2], staged);
}

}  // namespace render
}  // namespace lgs
