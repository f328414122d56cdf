// Shared host/device helpers of the gfx950 rasterizer library.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>

#include "localgs.h"

namespace lgs {

constexpr int kTile = LGS_TILE;          // 16x16 pixel tiles
constexpr int kBlock = 256;              // one workgroup per tile: 4 wave64
constexpr int kMaxViews = LGS_MAX_VIEWS; // cameras per view batch
constexpr int kL1Parts = 2048;            // partial sums of the L1 loss reduction
constexpr float kAlphaMax = 0.99f;       // opacity clamp (Sec. III-D-1)
constexpr double kTMin = 1e-4;           // termination threshold (Alg. 1)
constexpr double kLowpass = 0.3;         // 2D covariance dilation, px^2
constexpr double kGuard = 1.3;           // Jacobian evaluated inside 1.3x the frustum
// projected splat record: float4 (a, b, c, o), float4 (x, y, r, g), float b
// at float 8, zero padding; one 64-byte sector per element.  Gradient
// record: the same nine floats, packed.
constexpr int kSplatF = LGS_SPLAT_FLOATS;
constexpr int kSplatV = kSplatF / 4;     // float4 slots per record
constexpr int kGradF = LGS_GRAD_FLOATS;
static_assert(kSplatF == 16 && kGradF == 9, "record layouts");
constexpr double kLog2e = 1.4426950408889634074;
constexpr double kLn2 = 0.6931471805599453094;
// Footprint slack: tiles are assigned for the ellipse q <= tau*(1+rel)+abs,
// widened by kFootPx pixels, so the rectangle is conservative for any pixel
// whose alpha the render kernels keep.
constexpr double kFootRel = 1e-5;
constexpr double kFootAbs = 1e-5;
constexpr double kFootPx = 1e-2;

// ---------------------------------------------------------------------------
// error reporting (thread-local message)
// ---------------------------------------------------------------------------
void set_error(const char *fmt, ...);
lgs_status launch_status(const char *what);

#define LGS_REQUIRE(cond, ...)                                                    \
    do {                                                                          \
        if (!(cond)) {                                                            \
            ::lgs::set_error(__VA_ARGS__);                                        \
            return LGS_ERR_INVALID_ARG;                                           \
        }                                                                         \
    } while (0)

#define LGS_HIP(call)                                                             \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess) {                                                   \
            ::lgs::set_error("%s: %s", #call, hipGetErrorString(e_));             \
            return LGS_ERR_HIP;                                                   \
        }                                                                         \
    } while (0)

#define LGS_LAUNCHED(what)                                                        \
    do {                                                                          \
        lgs_status s_ = ::lgs::launch_status(what);                               \
        if (s_ != LGS_OK) return s_;                                              \
    } while (0)

// ---------------------------------------------------------------------------
// camera as passed to kernels (by value)
// ---------------------------------------------------------------------------
struct Cam {
    float view[12];
    float campos[3];
    float fx, fy, cx, cy;
    float tanx, tany;
    int W, H;
    float znear;
    float bg[3];
    int tiles_x, tiles_y;
};

inline bool cam_from(const lgs_camera *c, Cam &d)
{
    if (!c || c->width < 1 || c->height < 1) return false;
    if (c->width > (1 << 16) || c->height > (1 << 16)) return false;
    for (int i = 0; i < 12; ++i) d.view[i] = c->viewmat[i];
    for (int i = 0; i < 3; ++i) { d.campos[i] = c->campos[i]; d.bg[i] = c->bg[i]; }
    d.fx = c->fx; d.fy = c->fy; d.cx = c->cx; d.cy = c->cy;
    d.tanx = c->tan_fovx; d.tany = c->tan_fovy;
    d.W = c->width; d.H = c->height; d.znear = c->znear;
    d.tiles_x = (c->width + kTile - 1) / kTile;
    d.tiles_y = (c->height + kTile - 1) / kTile;
    return std::isfinite(d.fx) && std::isfinite(d.fy) && d.fx > 0 && d.fy > 0;
}

inline unsigned grid_for(int64_t n, int per_block) { return (unsigned)((n + per_block - 1) / per_block); }

// compute units of the current device (cached per device; 256 if unknown)
inline int device_cus()
{
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cached[dev] == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        cached[dev] = cus;
    }
    return cached[dev];
}

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << __lane_id()) - 1ull; }

// record e of a splat (or gradient) record array
__device__ __forceinline__ const float4 *splat_rec(const float *s, uint64_t e)
{
    return reinterpret_cast<const float4 *>(s) + e * kSplatV;
}

__device__ __forceinline__ float4 *splat_rec(float *s, uint64_t e)
{
    return reinterpret_cast<float4 *>(s) + e * kSplatV;
}

// the whole record as four 16-byte stores (one full sector)
__device__ __forceinline__ void store_splat(float *s, uint64_t e, float4 co, float4 mr, float b)
{
    float4 *r = splat_rec(s, e);
    r[0] = co;
    r[1] = mr;
    r[2] = make_float4(b, 0.f, 0.f, 0.f);
    r[3] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// fill kernel used instead of hipMemsetAsync so that every clear is an
// ordinary kernel node (graph-capture friendly)
template <typename T>
__global__ void fill_kernel(T *p, T v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

template <typename T>
inline void fill_async(T *p, T v, int64_t n, hipStream_t s)
{
    if (n <= 0) return;
    unsigned g = grid_for(n, 256);
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(fill_kernel<T>, dim3(g), dim3(256), 0, s, p, v, n);
}

}  // namespace lgs
