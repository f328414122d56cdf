// Preprocessing: projection of 3D Gaussians to screen-space splats, and its
// gradient.  Sec. II-A / Fig. 2 of the paper (preprocessing stage, inherited
// unchanged from 3DGS).  The stage streams the raw parameters once from HBM,
// so its geometry runs in double precision at no cost in throughput on
// gfx950 (full-rate FP64 FMA).
#include "common.hpp"

#include <type_traits>

namespace lgs {
namespace {

// real SH constants (Condon-Shortley phase), as closed forms
constexpr double kPi = 3.14159265358979323846;
__device__ __forceinline__ double sq(double x) { return x * x; }

// (in the precision T of the evaluation: double, or float for the colour)
template <typename T>
struct ShConst {
    T k0, k1, k2a, k2b, k2c, k3a, k3b, k3c, k3d, k3e;
};
template <typename T>
__device__ __forceinline__ ShConst<T> sh_consts()
{
    ShConst<T> k;
    k.k0 = (T)(0.5 / sqrt(kPi));               // Y_0^0
    k.k1 = (T)sqrt(3.0 / (4.0 * kPi));         // degree 1
    k.k2a = (T)(0.5 * sqrt(15.0 / kPi));       // xy, yz, xz terms
    k.k2b = (T)(0.25 * sqrt(5.0 / kPi));       // 3z^2 - 1
    k.k2c = (T)(0.25 * sqrt(15.0 / kPi));      // x^2 - y^2
    k.k3a = (T)(0.25 * sqrt(35.0 / (2.0 * kPi)));
    k.k3b = (T)(0.5 * sqrt(105.0 / kPi));
    k.k3c = (T)(0.25 * sqrt(21.0 / (2.0 * kPi)));
    k.k3d = (T)(0.25 * sqrt(7.0 / kPi));
    k.k3e = (T)(0.25 * sqrt(105.0 / kPi));
    return k;
}

// SH basis in index order l*l + l + m (m = -l..l) at unit direction (x, y, z).
template <int DEG, typename T>
__device__ __forceinline__ void sh_eval(T x, T y, T z, T *Y)
{
    const ShConst<T> k = sh_consts<T>();
    Y[0] = k.k0;
    if (DEG >= 1) {
        Y[1] = -k.k1 * y; Y[2] = k.k1 * z; Y[3] = -k.k1 * x;
    }
    if (DEG >= 2) {
        Y[4] = k.k2a * x * y;
        Y[5] = -k.k2a * y * z;
        Y[6] = k.k2b * ((T)3 * z * z - (T)1);
        Y[7] = -k.k2a * x * z;
        Y[8] = k.k2c * (x * x - y * y);
    }
    if (DEG >= 3) {
        const T zz5 = (T)5 * z * z - (T)1;
        Y[9] = -k.k3a * y * ((T)3 * x * x - y * y);
        Y[10] = k.k3b * x * y * z;
        Y[11] = -k.k3c * y * zz5;
        Y[12] = k.k3d * z * ((T)5 * z * z - (T)3);
        Y[13] = -k.k3c * x * zz5;
        Y[14] = k.k3e * z * (x * x - y * y);
        Y[15] = -k.k3a * x * (x * x - (T)3 * y * y);
    }
}

// g = sum_k w(k) grad Y_k at (x, y, z): the weighted gradient of the basis,
// accumulated term by term so that no per-basis gradient table is held; the
// weights come from a callable, evaluated where each is used (no table of
// them either).
template <int DEG, typename T, typename WF>
__device__ __forceinline__ void sh_grad_dir(T x, T y, T z, WF &&wf, T *g)
{
    T w[16];
#pragma unroll
    for (int k = 1; k < (DEG + 1) * (DEG + 1); ++k) w[k] = wf(k);
    const ShConst<T> k = sh_consts<T>();
    T gx = 0, gy = 0, gz = 0;
    if (DEG >= 1) {
        gy -= k.k1 * w[1];
        gz += k.k1 * w[2];
        gx -= k.k1 * w[3];
    }
    if (DEG >= 2) {
        gx += k.k2a * y * w[4]; gy += k.k2a * x * w[4];
        gy -= k.k2a * z * w[5]; gz -= k.k2a * y * w[5];
        gz += (T)6 * k.k2b * z * w[6];
        gx -= k.k2a * z * w[7]; gz -= k.k2a * x * w[7];
        gx += (T)2 * k.k2c * x * w[8]; gy -= (T)2 * k.k2c * y * w[8];
    }
    if (DEG >= 3) {
        const T zz5 = (T)5 * z * z - (T)1, d33 = (T)3 * x * x - (T)3 * y * y, xy6 = (T)6 * x * y;
        gx -= k.k3a * xy6 * w[9]; gy -= k.k3a * d33 * w[9];
        gx += k.k3b * y * z * w[10]; gy += k.k3b * x * z * w[10]; gz += k.k3b * x * y * w[10];
        gy -= k.k3c * zz5 * w[11]; gz -= k.k3c * (T)10 * y * z * w[11];
        gz += k.k3d * ((T)15 * z * z - (T)3) * w[12];
        gx -= k.k3c * zz5 * w[13]; gz -= k.k3c * (T)10 * x * z * w[13];
        gx += (T)2 * k.k3e * x * z * w[14]; gy -= (T)2 * k.k3e * y * z * w[14]; gz += k.k3e * (x * x - y * y) * w[14];
        gx -= k.k3a * d33 * w[15]; gy += k.k3a * xy6 * w[15];
    }
    g[0] = gx; g[1] = gy; g[2] = gz;
}

// Forward intermediates of one Gaussian, kept for the backward recompute.
struct Proj {
    bool visible;
    double m[3], s[3], o;
    double t[3];
    double R[3][3];
    double TM[2][3];         // T M with M = R diag(s): Sigma2 = TM TM^T + low-pass
    double u, v;             // clamped tangent-plane coordinates
    bool uc, vc;             // clamp active
    double J00, J02, J11, J12;
    double T[2][3];
    double X, Y, Z;          // Sigma2 xx, yy, xy (with the low-pass)
    double det;
    double a, b, c;          // conic
    double mx, my;           // projected mean
    double tau;              // footprint level 2 ln(255 o)
};

// true if none of the k floats is inf or NaN (exponent bits all ones), with
// no early exit so that the check stays branch-free
__device__ __forceinline__ bool all_finite(const float *p, int k)
{
    uint32_t bad = 0;
    for (int i = 0; i < k; ++i) bad |= ((__float_as_uint(p[i]) & 0x7f800000u) == 0x7f800000u) ? 1u : 0u;
    return bad == 0;
}

// The view-independent part of a Gaussian's projection: finiteness of its
// parameters, the normalised quaternion, the scales, the opacity and the
// footprint level tau = 2 ln(255 o); computed once per Gaussian and reused
// for every view of a batch (each is a transcendental in double).
struct GaussPre {
    bool ok;                 // parameters finite and quaternion nonzero
    double qn[4], qlen, s[3], o, tau;
};

__device__ __forceinline__ GaussPre gauss_pre(const float *m3, const float *ls, const float *qt, float logit)
{
    GaussPre g;
    g.ok = all_finite(m3, 3) & all_finite(ls, 3) & all_finite(qt, 4) & all_finite(&logit, 1);
    const double q0 = qt[0], q1 = qt[1], q2 = qt[2], q3 = qt[3];
    const double n2 = q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3;
    g.ok = g.ok && n2 > 0.0;
    g.qlen = sqrt(n2);
    const double inv = 1.0 / g.qlen;
    g.qn[0] = q0 * inv; g.qn[1] = q1 * inv; g.qn[2] = q2 * inv; g.qn[3] = q3 * inv;
    for (int j = 0; j < 3; ++j) g.s[j] = exp((double)ls[j]);
    g.o = 1.0 / (1.0 + exp(-(double)logit));
    g.tau = 2.0 * log(255.0 * g.o);
    return g;
}

// rotation matrix of the unit quaternion (w, x, y, z)
__device__ __forceinline__ void rotation(const double *qn, double (&R)[3][3])
{
    const double w = qn[0], x = qn[1], y = qn[2], z = qn[3];
    R[0][0] = 1.0 - 2.0 * (y * y + z * z); R[0][1] = 2.0 * (x * y - w * z); R[0][2] = 2.0 * (x * z + w * y);
    R[1][0] = 2.0 * (x * y + w * z); R[1][1] = 1.0 - 2.0 * (x * x + z * z); R[1][2] = 2.0 * (y * z - w * x);
    R[2][0] = 2.0 * (x * z - w * y); R[2][1] = 2.0 * (y * z + w * x); R[2][2] = 1.0 - 2.0 * (x * x + y * y);
}

// Geometry of the projection (no colour) for one view.  Returns false if
// culled before the footprint test.
__device__ bool project_geometry(const Cam &cam, const float *m3, const GaussPre &G, Proj &P)
{
    if (!G.ok) return false;
    const float *V = cam.view;
    for (int i = 0; i < 3; ++i) P.m[i] = m3[i];
    // camera-space position; this FMA order defines the depth key
    for (int k = 0; k < 3; ++k)
        P.t[k] = fma((double)V[4 * k + 2], P.m[2], fma((double)V[4 * k + 1], P.m[1],
                 fma((double)V[4 * k + 0], P.m[0], (double)V[4 * k + 3])));
    if (!(P.t[2] > (double)cam.znear)) return false;
    rotation(G.qn, P.R);
    for (int j = 0; j < 3; ++j) P.s[j] = G.s[j];
    const double fx = cam.fx, fy = cam.fy;
    const double limx = kGuard * (double)cam.tanx, limy = kGuard * (double)cam.tany;
    const double tz = P.t[2], rz = 1.0 / tz;
    double u = P.t[0] * rz, v = P.t[1] * rz;
    P.uc = false; P.vc = false;
    if (u < -limx) { u = -limx; P.uc = true; } else if (u > limx) { u = limx; P.uc = true; }
    if (v < -limy) { v = -limy; P.vc = true; } else if (v > limy) { v = limy; P.vc = true; }
    P.u = u; P.v = v;
    P.J00 = fx * rz; P.J02 = -fx * u * rz; P.J11 = fy * rz; P.J12 = -fy * v * rz;
    for (int j = 0; j < 3; ++j) {
        P.T[0][j] = P.J00 * (double)V[0 * 4 + j] + P.J02 * (double)V[2 * 4 + j];
        P.T[1][j] = P.J11 * (double)V[1 * 4 + j] + P.J12 * (double)V[2 * 4 + j];
    }
    // Sigma2 = T Sigma3 T^T + low-pass with Sigma3 = M M^T: Sigma2 = (T M)(T M)^T
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j)
            P.TM[i][j] = (P.T[i][0] * P.R[0][j] + P.T[i][1] * P.R[1][j] + P.T[i][2] * P.R[2][j]) * P.s[j];
    P.X = P.TM[0][0] * P.TM[0][0] + P.TM[0][1] * P.TM[0][1] + P.TM[0][2] * P.TM[0][2] + kLowpass;
    P.Y = P.TM[1][0] * P.TM[1][0] + P.TM[1][1] * P.TM[1][1] + P.TM[1][2] * P.TM[1][2] + kLowpass;
    P.Z = P.TM[0][0] * P.TM[1][0] + P.TM[0][1] * P.TM[1][1] + P.TM[0][2] * P.TM[1][2];
    P.det = P.X * P.Y - P.Z * P.Z;
    if (!(P.det > 0.0)) return false;
    const double id = 1.0 / P.det;
    P.a = P.Y * id; P.b = -P.Z * id; P.c = P.X * id;
    P.mx = fx * P.t[0] * rz + (double)cam.cx;
    P.my = fy * P.t[1] * rz + (double)cam.cy;
    P.o = G.o;
    P.tau = G.tau;
    return true;
}

// Unit view direction (mean - camera centre) in single precision, for the SH
// colour, and 1 / |mean - camera centre| (0 for a mean on the centre, whose
// direction is taken as +z).  Each difference of two floats is exact to
// within one rounding, so every component is within a few units in the last
// place of its value.
struct ViewDir {
    float x, y, z, il;
};
__device__ __forceinline__ ViewDir view_dir(const Cam &cam, const float *m3)
{
    const float d0 = m3[0] - cam.campos[0], d1 = m3[1] - cam.campos[1], d2 = m3[2] - cam.campos[2];
    const float s2 = d0 * d0 + d1 * d1 + d2 * d2;
    ViewDir d;
    d.il = s2 > 0.f ? rsqrtf(s2) : 0.f;
    d.x = d0 * d.il; d.y = d1 * d.il; d.z = s2 > 0.f ? d2 * d.il : 1.f;
    return d;
}


// Tile rectangle of the footprint; false if it covers no pixel centre.
__device__ bool footprint(const Cam &cam, const Proj &P, int4 &rect)
{
    const double tau = P.tau;
    if (!(tau > 0.0)) return false;
    double tm = tau * (1.0 + kFootRel) + kFootAbs;
    double rx = sqrt(tm * P.X) + kFootPx, ry = sqrt(tm * P.Y) + kFootPx;
    double x0 = ceil(P.mx - rx), x1 = floor(P.mx + rx), y0 = ceil(P.my - ry), y1 = floor(P.my + ry);
    if (!(isfinite(x0) && isfinite(x1) && isfinite(y0) && isfinite(y1))) return false;
    x0 = fmax(x0, 0.0); y0 = fmax(y0, 0.0);
    x1 = fmin(x1, (double)(cam.W - 1)); y1 = fmin(y1, (double)(cam.H - 1));
    if (x0 > x1 || y0 > y1) return false;
    rect.x = (int)x0 / kTile; rect.y = (int)y0 / kTile;
    rect.z = (int)x1 / kTile + 1; rect.w = (int)y1 / kTile + 1;
    return true;
}

// LDS row stride of one Gaussian's 3K SH floats: odd, so that the 64 lanes
// reading "their" coefficient k hit distinct banks (a stride of 48 words
// would put all lanes on two banks).
constexpr int sh_stride(int K3) { return K3 | 1; }

// Wavefront-cooperative copy of the SH coefficients of this wavefront's 64
// Gaussians (one contiguous run of 64 * 3K floats) into LDS rows of
// sh_stride(3K) floats, with 16-byte loads, so that no lane reads its own
// strided record from HBM.
template <int K3>
__device__ __forceinline__ void stage_sh(const float *__restrict__ sh, int64_t g0, int cnt, float *s_sh)
{
    constexpr int P = sh_stride(K3);
    const float *src = sh + g0 * K3;
    const int total = cnt * K3;
    const int nv = total >> 2;
    const float4 *src4 = reinterpret_cast<const float4 *>(src);
    if constexpr (P == K3) {
        float4 *dst4 = reinterpret_cast<float4 *>(s_sh);
        for (int i = __lane_id(); i < nv; i += 64) dst4[i] = src4[i];
    } else {
        for (int i = __lane_id(); i < nv; i += 64) {
            const float4 v = src4[i];
            const int e = 4 * i, g = e / K3, k = e - g * K3;      // K3 % 4 == 0: one row
            float *d = s_sh + g * P + k;
            d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w;
        }
    }
    for (int i = (nv << 2) + __lane_id(); i < total; i += 64) s_sh[(i / K3) * P + i % K3] = src[i];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Splat records of a wavefront's 64 Gaussians, stored by groups of eight
// lanes so that every store instruction writes whole 128-byte lines.  First
// the four lanes of a quad transpose their records' 16-byte quarters among
// themselves (two butterfly stages over lane ^ 1 and lane ^ 2): lane p of quad
// b then holds quarter p of records 4b .. 4b + 3.  Then the two quads of a
// group exchange two quarters (lane ^ 4), after which store s writes records
// 2s and 2s + 1 of every group, lanes 0-3 the one and lanes 4-7 the other.
// All 64 lanes take part (a record of zeros for lanes past the end, which
// store nothing).
template <int CTRL>
__device__ __forceinline__ float quad_read(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// one butterfly exchange over the lane pair (p, p ^ m): of the pair of
// quarters (a, b), a lane whose bit m is clear keeps a and receives the
// partner's a into b; the other keeps b and receives the partner's b into a
template <int CTRL>
__device__ __forceinline__ void quad_swap(float &a, float &b, bool hi)
{
    const float r = quad_read<CTRL>(hi ? a : b);
    a = hi ? r : a;
    b = hi ? b : r;
}

// the value of lane ^ 4 (within each group of 32 lanes: swizzle, xor mask 4)
__device__ __forceinline__ float xor4_read(float v)
{
    return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x1F | (4 << 10)));
}

// grp: index of the group's first record (from the wavefront's base, not
// from a lane's own index, which is clamped for lanes past the end)
__device__ __forceinline__ void store_splats_oct(float *s, uint64_t grp, uint32_t oct_in, float4 co, float4 mr,
                                                 float bl)
{
    const int l8 = __lane_id() & 7, p = l8 & 3;
    float q[4][4] = {{co.x, co.y, co.z, co.w}, {mr.x, mr.y, mr.z, mr.w}, {bl, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
    // quad transpose, stage 1 over lane ^ 1: quarters (0, 1) and (2, 3) (of
    // those only the first components are nonzero)
    const bool h1 = (p & 1) != 0, h2 = (p & 2) != 0, c1 = l8 >= 4;
#pragma unroll
    for (int c = 0; c < 4; ++c) quad_swap<0xB1>(q[0][c], q[1][c], h1);    // quad_perm [1,0,3,2]
    quad_swap<0xB1>(q[2][0], q[3][0], h1);
    // stage 2 over lane ^ 2: quarters (0, 2) and (1, 3)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        quad_swap<0x4E>(q[0][c], q[2][c], h2);                            // quad_perm [2,3,0,1]
        quad_swap<0x4E>(q[1][c], q[3][c], h2);
    }
    // lane p of quad b now holds quarter p of records 4b + j in q[j]; the
    // first quad of a group (c1 clear) sends q[1], q[3] and takes the second
    // one's q[0], q[2]
    float x[4], y[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        x[c] = xor4_read(c1 ? q[0][c] : q[1][c]);
        y[c] = xor4_read(c1 ? q[2][c] : q[3][c]);
    }
    float4 *base = splat_rec(s, grp);                                    // record 0 of the group
    float4 out[4];
    out[0] = c1 ? make_float4(x[0], x[1], x[2], x[3]) : make_float4(q[0][0], q[0][1], q[0][2], q[0][3]);
    out[1] = c1 ? make_float4(y[0], y[1], y[2], y[3]) : make_float4(q[2][0], q[2][1], q[2][2], q[2][3]);
    out[2] = c1 ? make_float4(q[1][0], q[1][1], q[1][2], q[1][3]) : make_float4(x[0], x[1], x[2], x[3]);
    out[3] = c1 ? make_float4(q[3][0], q[3][1], q[3][2], q[3][3]) : make_float4(y[0], y[1], y[2], y[3]);
    // store s: record 2s + c1 of the group, quarter p (oct_in: bit k set if
    // the group's lane k has a Gaussian)
    const int c = c1 ? 1 : 0;
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4)
        if ((oct_in >> (2 * s4 + c)) & 1u) base[(2 * s4 + c) * kSplatV + p] = out[s4];
}

// cameras of a view batch, passed by value as a kernel argument
struct CamBatch {
    Cam cam[kMaxViews];
    int V;
};

// Projection of n Gaussians for every camera of the batch: the raw
// parameters (and the SH coefficients, staged in LDS) are read once and
// projected V times; outputs are view-major, element v * n + i.
template <int DEG>
__global__ __launch_bounds__(256) void project_fwd_kernel(CamBatch cb, int64_t n, const float *__restrict__ means3d,
                                                          const float *__restrict__ log_scales,
                                                          const float *__restrict__ quats,
                                                          const float *__restrict__ logits,
                                                          const float *__restrict__ sh, float *__restrict__ splats,
                                                          float *__restrict__ depth, int4 *__restrict__ rect)
{
    constexpr int K = (DEG + 1) * (DEG + 1);
    __shared__ float s_sh[4][64 * sh_stride(3 * K)];
    const int wid = threadIdx.x >> 6;
    const int64_t g0 = (int64_t)blockIdx.x * blockDim.x + wid * 64;
    if (g0 >= n) return;                                   // whole wavefront past the end
    stage_sh<3 * K>(sh, g0, (int)min((int64_t)64, n - g0), s_sh[wid]);
    // every lane of the wavefront stays to the end (the records are stored
    // by groups of lanes); a lane past the end computes on its wavefront's
    // first Gaussian and stores nothing
    const bool in = g0 + __lane_id() < n;
    const int64_t i = in ? g0 + __lane_id() : g0;
    const uint32_t oct_in = (uint32_t)(__ballot(in) >> (__lane_id() & ~7u)) & 0xFFu;
    const float m3[3] = {means3d[3 * i], means3d[3 * i + 1], means3d[3 * i + 2]};
    const float ls[3] = {log_scales[3 * i], log_scales[3 * i + 1], log_scales[3 * i + 2]};
    const float4 q4 = reinterpret_cast<const float4 *>(quats)[i];
    const float qt[4] = {q4.x, q4.y, q4.z, q4.w};
    const float logit = logits[i];
    const float *shi = s_sh[wid] + (in ? __lane_id() : 0) * sh_stride(3 * K);
    const bool sh_ok = all_finite(shi, 3 * K);
    const GaussPre G = gauss_pre(m3, ls, qt, logit);
    for (int v = 0; v < cb.V; ++v) {
        const Cam &cam = cb.cam[v];
        const int64_t o = (int64_t)v * n + i;
        Proj P;
        int4 r = make_int4(0, 0, 0, 0);
        const bool vis = sh_ok && project_geometry(cam, m3, G, P) && footprint(cam, P, r);
        // culled: an all-zero record, depth +inf and an empty rectangle
        float4 co = make_float4(0.f, 0.f, 0.f, 0.f), mr = co;
        float bl = 0.f, dz = INFINITY;
        if (vis) {
            // colour in single precision (a continuous function of the
            // sum: its error bound is kColourTol's)
            const ViewDir d = view_dir(cam, m3);
            float Y[K];
            sh_eval<DEG>(d.x, d.y, d.z, Y);
            float col[3] = {0.5f, 0.5f, 0.5f};
#pragma unroll
            for (int k = 0; k < K; ++k) {
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) col[ch] = fmaf(shi[3 * k + ch], Y[k], col[ch]);
            }
            co = make_float4((float)P.a, (float)P.b, (float)P.c, (float)P.o);
            mr = make_float4((float)P.mx, (float)P.my, fmaxf(col[0], 0.f), fmaxf(col[1], 0.f));
            bl = fmaxf(col[2], 0.f);
            dz = (float)P.t[2];
        } else {
            r = make_int4(0, 0, 0, 0);
        }
        store_splats_oct(splats, (uint64_t)v * n + g0 + (__lane_id() & ~7u), oct_in, co, mr, bl);
        if (in) {
            depth[o] = dz;
            rect[o] = r;
        }
    }
}

// One view's gradient of a Gaussian: of the mean, of the opacity logit, and
// of M = R diag(s) (the scales and the quaternion depend on the view only
// through M, and linearly in dL/dM, so their chain is applied once to the sum
// over views: rot_scale_grad).
struct RawGrad {
    double m[3], M[3][3], logit;
};
constexpr int kRawGradD = 13;   // doubles in a RawGrad

// dL/d log-scales and dL/d raw quaternion from dL/dM summed over views:
// M = R diag(s) with s = exp(log-scales) and R the rotation of q / |q|.
__device__ __forceinline__ void rot_scale_grad(const GaussPre &G, const double (&gM)[3][3], double *gls,
                                               double *gqr)
{
    double R[3][3];
    rotation(G.qn, R);
    // dL/dR[a][b] = dL/dM[a][b] s[b], dL/ds[b] = sum_a dL/dM[a][b] R[a][b]
    double gR[3][3], gs[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            gR[a][b] = gM[a][b] * G.s[b];
            gs[b] += gM[a][b] * R[a][b];
        }
    for (int k = 0; k < 3; ++k) gls[k] = gs[k] * G.s[k];
    // through the rotation matrix of the unit quaternion
    const double w = G.qn[0], x = G.qn[1], y = G.qn[2], z = G.qn[3];
    double gq[4];
    gq[0] = 2.0 * (-z * gR[0][1] + y * gR[0][2] + z * gR[1][0] - x * gR[1][2] - y * gR[2][0] + x * gR[2][1]);
    gq[1] = 2.0 * (y * gR[0][1] + z * gR[0][2] + y * gR[1][0] - 2.0 * x * gR[1][1] - w * gR[1][2] + z * gR[2][0]
                   + w * gR[2][1] - 2.0 * x * gR[2][2]);
    gq[2] = 2.0 * (-2.0 * y * gR[0][0] + x * gR[0][1] + w * gR[0][2] + x * gR[1][0] + z * gR[1][2] - w * gR[2][0]
                   + z * gR[2][1] - 2.0 * y * gR[2][2]);
    gq[3] = 2.0 * (-2.0 * z * gR[0][0] - w * gR[0][1] + x * gR[0][2] + w * gR[1][0] - 2.0 * z * gR[1][1]
                   + y * gR[1][2] + x * gR[2][0] + y * gR[2][1]);
    // normalisation q / |q|
    const double dq = gq[0] * w + gq[1] * x + gq[2] * y + gq[3] * z;
    const double iq = 1.0 / G.qlen;
    gqr[0] = (gq[0] - w * dq) * iq;
    gqr[1] = (gq[1] - x * dq) * iq;
    gqr[2] = (gq[2] - y * dq) * iq;
    gqr[3] = (gq[3] - z * dq) * iq;
}

// One view's contribution of a Gaussian whose projected attributes received
// a gradient.  m3 is its mean, G its view-independent terms, shi its SH
// coefficients and dshi[k * dstride] the LDS accumulators of dL/d sh: double
// ones are added to atomically (several views of one Gaussian may be taken at
// once), float ones belong to the calling lane alone.  g* are this view's
// gradients of the projected attributes.  The SH gradient is always added;
// the rest is written to out (added to it with float accumulators, whose
// caller sums over views in registers) only if the projection's geometry is
// valid, which the return value says.
template <int DEG, typename ACC>
__device__ __forceinline__ bool project_bwd_view(const Cam &cam, const float *m3, const GaussPre &G,
                                                 const float *shi, const float2 g2, const float *g_con, float g_op,
                                                 const float *g_col, RawGrad &out, ACC *dshi, int dstride)
{
    constexpr int K = (DEG + 1) * (DEG + 1);
    // The colour's gradient first: it needs only the view direction, so its
    // basis and weights are dead before the projection's intermediates are
    // recomputed below (fewer registers live at once).
    double gm[3] = {0.0, 0.0, 0.0};
    {
        const double d0 = (double)m3[0] - (double)cam.campos[0], d1 = (double)m3[1] - (double)cam.campos[1],
                     d2 = (double)m3[2] - (double)cam.campos[2];
        const double dlen = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        double dir[3] = {0.0, 0.0, 1.0};
        const double il = dlen > 0.0 ? 1.0 / dlen : 0.0;
        if (dlen > 0.0) { dir[0] = d0 * il; dir[1] = d1 * il; dir[2] = d2 * il; }
        double gcol[3] = {g_col[0], g_col[1], g_col[2]};
        // colour: rgb = max(0, sum_k sh_k Y_k(dir) + 0.5)
        double Y[K];
        sh_eval<DEG>(dir[0], dir[1], dir[2], Y);
        for (int ch = 0; ch < 3; ++ch) {
            double val = 0.5;
            for (int k = 0; k < K; ++k) val += (double)shi[3 * k + ch] * Y[k];
            if (val < 0.0) gcol[ch] = 0.0;
        }
        // re-read the coefficients from LDS below rather than keeping all 3K
        // of them in registers across the passes (a compiler barrier only)
        __asm__ volatile("" ::: "memory");
        for (int k = 0; k < K; ++k)
            for (int ch = 0; ch < 3; ++ch) {
                if constexpr (std::is_same<ACC, double>::value) atomicAdd(&dshi[(3 * k + ch) * dstride], gcol[ch] * Y[k]);
                else dshi[(3 * k + ch) * dstride] += (float)(gcol[ch] * Y[k]);
            }
        // dL/d dir = sum_k (sum_ch gcol_ch sh_k,ch) grad Y_k
        double gdir[3];
        sh_grad_dir<DEG>(dir[0], dir[1], dir[2], [&](int k) {
            return gcol[0] * (double)shi[3 * k] + gcol[1] * (double)shi[3 * k + 1] + gcol[2] * (double)shi[3 * k + 2];
        }, gdir);
        if (dlen > 0.0) {
            const double dd = gdir[0] * dir[0] + gdir[1] * dir[1] + gdir[2] * dir[2];
            for (int k = 0; k < 3; ++k) gm[k] += (gdir[k] - dir[k] * dd) * il;
        }
    }
    Proj P;
    if (!project_geometry(cam, m3, G, P)) return false;
    const double gmx = g2.x, gmy = g2.y;
    const double ga = g_con[0], gb = g_con[1], gc = g_con[2];
    const double go = g_op;

    // opacity = sigmoid(logit)
    constexpr bool kAdd = !std::is_same<ACC, double>::value;
    const double glogit = go * P.o * (1.0 - P.o);
    out.logit = kAdd ? out.logit + glogit : glogit;

    // conic (a, b, c) = (Y, -Z, X) / det  ->  Sigma2 entries X, Y, Z
    const double id = 1.0 / P.det, id2 = id * id;
    const double gX = ga * (-P.Y * P.Y * id2) + gb * (P.Z * P.Y * id2) + gc * (id - P.X * P.Y * id2);
    const double gY = ga * (id - P.Y * P.X * id2) + gb * (P.Z * P.X * id2) + gc * (-P.X * P.X * id2);
    const double gZ = ga * (2.0 * P.Y * P.Z * id2) + gb * (-id - 2.0 * P.Z * P.Z * id2) + gc * (2.0 * P.X * P.Z * id2);
    // symmetric gradient of Sigma2 = TM TM^T (+ low-pass), TM = T M:
    // dL/dTM = 2 G2 TM, then dL/dT = dL/dTM M^T and dL/dM = T^T dL/dTM
    const double G2[2][2] = {{gX, 0.5 * gZ}, {0.5 * gZ, gY}};
    double gTM[2][3];
    for (int i2 = 0; i2 < 2; ++i2)
        for (int j = 0; j < 3; ++j) gTM[i2][j] = 2.0 * (G2[i2][0] * P.TM[0][j] + G2[i2][1] * P.TM[1][j]);
    double gT[2][3];
    for (int i2 = 0; i2 < 2; ++i2)
        for (int k = 0; k < 3; ++k)
            gT[i2][k] = gTM[i2][0] * P.R[k][0] * P.s[0] + gTM[i2][1] * P.R[k][1] * P.s[1]
                        + gTM[i2][2] * P.R[k][2] * P.s[2];
    // T = J W: dL/dJ[i][k] = sum_j gT[i][j] W[k][j]
    const float *V = cam.view;
    double gJ00 = 0, gJ02 = 0, gJ11 = 0, gJ12 = 0;
    for (int j = 0; j < 3; ++j) {
        gJ00 += gT[0][j] * (double)V[0 * 4 + j];
        gJ02 += gT[0][j] * (double)V[2 * 4 + j];
        gJ11 += gT[1][j] * (double)V[1 * 4 + j];
        gJ12 += gT[1][j] * (double)V[2 * 4 + j];
    }
    const double fx = cam.fx, fy = cam.fy, tx = P.t[0], ty = P.t[1], tz = P.t[2];
    const double rz = 1.0 / tz, rz2 = rz * rz;
    double gt[3] = {0.0, 0.0, 0.0};
    // J00 = fx/tz, J11 = fy/tz
    gt[2] += gJ00 * (-fx * rz2) + gJ11 * (-fy * rz2);
    // J02 = -fx u / tz with u = tx/tz unless clamped
    if (!P.uc) { gt[0] += gJ02 * (-fx * rz2); gt[2] += gJ02 * (2.0 * fx * tx * rz2 * rz); }
    else gt[2] += gJ02 * (fx * P.u * rz2);
    if (!P.vc) { gt[1] += gJ12 * (-fy * rz2); gt[2] += gJ12 * (2.0 * fy * ty * rz2 * rz); }
    else gt[2] += gJ12 * (fy * P.v * rz2);
    // projected mean
    gt[0] += gmx * fx * rz; gt[2] += gmx * (-fx * tx * rz2);
    gt[1] += gmy * fy * rz; gt[2] += gmy * (-fy * ty * rz2);
    // t = W m + t_c
    for (int k = 0; k < 3; ++k)
        gm[k] += (double)V[0 * 4 + k] * gt[0] + (double)V[1 * 4 + k] * gt[1] + (double)V[2 * 4 + k] * gt[2];
    for (int k = 0; k < 3; ++k) out.m[k] = kAdd ? out.m[k] + gm[k] : gm[k];

    // dL/dM = T^T dL/dTM (rot_scale_grad applies the rest to the sum)
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            const double gM = P.T[0][a] * gTM[0][b] + P.T[1][a] * gTM[1][b];
            out.M[a][b] = kAdd ? out.M[a][b] + gM : gM;
        }
    return true;
}


// copy this wavefront's LDS slots back to HBM with 16-byte stores
template <int K3>
__device__ __forceinline__ void unstage_sh(float *__restrict__ dst_all, int64_t g0, int cnt, const float *s_sh)
{
    constexpr int P = sh_stride(K3);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float *dst = dst_all + g0 * K3;
    const int total = cnt * K3;
    const int nv = total >> 2;
    float4 *dst4 = reinterpret_cast<float4 *>(dst);
    if constexpr (P == K3) {
        const float4 *src4 = reinterpret_cast<const float4 *>(s_sh);
        for (int i = __lane_id(); i < nv; i += 64) dst4[i] = src4[i];
    } else {
        for (int i = __lane_id(); i < nv; i += 64) {
            const int e = 4 * i, g = e / K3, k = e - g * K3;
            const float *q = s_sh + g * P + k;
            dst4[i] = make_float4(q[0], q[1], q[2], q[3]);
        }
    }
    for (int i = (nv << 2) + __lane_id(); i < total; i += 64) dst[i] = s_sh[(i / K3) * P + i % K3];
}

// Backward of the projection for a batch of few views: one lane per
// Gaussian loops over the views (view v + 1's gradient record and rectangle
// loaded while view v is accumulated), with its sums in registers and its SH
// gradient in its own LDS row.  With few views a wavefront rarely has a view
// in which none of its Gaussians has a gradient, and listing the pairs
// (project_bwd_kernel below) would take as many rounds as this loop.
template <int DEG>
__global__ __launch_bounds__(128) void project_bwd_loop_kernel(
    CamBatch cb, int64_t n, const float *__restrict__ means3d, const float *__restrict__ log_scales,
    const float *__restrict__ quats, const float *__restrict__ logits, const float *__restrict__ sh,
    const int4 *__restrict__ rect, float *__restrict__ g_splats, bool clear, float *__restrict__ d_means3d,
    float *__restrict__ d_log_scales, float *__restrict__ d_quats, float *__restrict__ d_logits,
    float *__restrict__ d_sh)
{
    constexpr int K3 = 3 * (DEG + 1) * (DEG + 1);
    constexpr int P = sh_stride(K3);
    __shared__ float s_sh[2][64 * P];
    __shared__ float s_dsh[2][64 * P];
    const int wid = threadIdx.x >> 6;
    const int64_t g0 = (int64_t)blockIdx.x * blockDim.x + wid * 64;
    if (g0 >= n) return;                                   // whole wavefront past the end
    const int cnt = (int)min((int64_t)64, n - g0);
    stage_sh<K3>(sh, g0, cnt, s_sh[wid]);
    const int64_t i = g0 + __lane_id();
    float *dslot = s_dsh[wid] + __lane_id() * P;
    for (int k = 0; k < K3; ++k) dslot[k] = 0.f;
    if (i < n) {
        const float m3[3] = {means3d[3 * i], means3d[3 * i + 1], means3d[3 * i + 2]};
        const float ls[3] = {log_scales[3 * i], log_scales[3 * i + 1], log_scales[3 * i + 2]};
        const float4 q4 = reinterpret_cast<const float4 *>(quats)[i];
        const float qt[4] = {q4.x, q4.y, q4.z, q4.w};
        const float *shi = s_sh[wid] + __lane_id() * P;
        const GaussPre G = gauss_pre(m3, ls, qt, logits[i]);
        RawGrad acc = {};
        float gn[kGradF];
        int4 rn;
        auto fetch = [&](int v) {
            const int64_t o = (int64_t)v * n + i;
            const float *gr = g_splats + (uint64_t)o * kGradF;
#pragma unroll
            for (int c = 0; c < kGradF; ++c) gn[c] = gr[c];
            rn = rect[o];
        };
        fetch(0);
        for (int v = 0; v < cb.V; ++v) {
            float gv[kGradF];
#pragma unroll
            for (int c = 0; c < kGradF; ++c) gv[c] = gn[c];
            const int4 rv = rn;
            if (v + 1 < cb.V) fetch(v + 1);
            bool nz = false;
#pragma unroll
            for (int c = 0; c < kGradF; ++c) nz = nz || gv[c] != 0.f;
            if (clear && nz) {
                // read and cleared: the record is zero for the next backward
                float *gr = g_splats + ((uint64_t)v * n + i) * kGradF;
#pragma unroll
                for (int c = 0; c < kGradF; ++c) gr[c] = 0.f;
            }
            // a view that sends no gradient (the Gaussian culled, or covered
            // by nearer ones in every pixel it reaches) adds nothing
            if (!(nz && rv.z > rv.x && rv.w > rv.y)) continue;
            const float gc3[3] = {gv[0], gv[1], gv[2]};
            const float gr3[3] = {gv[6], gv[7], gv[8]};
            project_bwd_view<DEG, float>(cb.cam[v], m3, G, shi, make_float2(gv[4], gv[5]), gc3, gv[3], gr3, acc, dslot,
                                         1);
        }
        double gls[3] = {0.0, 0.0, 0.0}, gq[4] = {0.0, 0.0, 0.0, 0.0};
        if (G.ok) rot_scale_grad(G, acc.M, gls, gq);
        for (int k = 0; k < 3; ++k) { d_means3d[3 * i + k] = (float)acc.m[k]; d_log_scales[3 * i + k] = (float)gls[k]; }
        for (int k = 0; k < 4; ++k) d_quats[4 * i + k] = (float)gq[k];
        d_logits[i] = (float)acc.logit;
    }
    unstage_sh<K3>(d_sh, g0, cnt, s_dsh[wid]);
}

// views up to which the backward projection loops over the views per
// Gaussian instead of listing the pairs (measured on a 10M-Gaussian training
// step: the loop is faster up to 8 views, 3.25 against 3.46 ms at 8; the
// list at 16, 4.33 against 5.55 ms)
constexpr int kLoopViews = 8;

// Row stride (in doubles) of the coefficient-major LDS accumulators of the
// SH gradient, [k][Gaussian]: 65, not 64, so that the transposing copy-out's
// lanes (consecutive coefficients of one Gaussian) fall in different banks.
constexpr int kDshStride = 65;

// copy a wavefront's coefficient-major SH gradient [k][Gaussian] to HBM,
// Gaussian-major, with 16-byte stores (the run of cnt * 3K floats starts
// 16-byte aligned: the wavefront's first Gaussian is a multiple of 64)
template <int K3>
__device__ __forceinline__ void unstage_dsh(float *__restrict__ dst_all, int64_t g0, int cnt, const double *s_dsh)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float *dst = dst_all + g0 * K3;
    auto at = [&](int e) { const int g = e / K3; return (float)s_dsh[(e - g * K3) * kDshStride + g]; };
    const int total = cnt * K3, nv = total >> 2;
    float4 *dst4 = reinterpret_cast<float4 *>(dst);
    for (int q = __lane_id(); q < nv; q += 64) dst4[q] = make_float4(at(4 * q), at(4 * q + 1), at(4 * q + 2), at(4 * q + 3));
    for (int e = (nv << 2) + __lane_id(); e < total; e += 64) dst[e] = at(e);
}

// the value x of lane src (src4 = 4 src), for 32- and 64-bit values
__device__ __forceinline__ float from_lane(float x, int src4)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src4, __float_as_int(x)));
}
__device__ __forceinline__ double from_lane(double x, int src4)
{
    const int lo = __builtin_amdgcn_ds_bpermute(src4, __double2loint(x));
    const int hi = __builtin_amdgcn_ds_bpermute(src4, __double2hiint(x));
    return __hiloint2double(hi, lo);
}

// Backward of the projection for a batch of views.  A workgroup of two
// wavefronts per 64 Gaussians (lane l of each holds Gaussian l's parameters).
// A Gaussian receives a gradient in few of the views (in a training step of
// 16 views over a dense scene, 17 % of the (Gaussian, view) pairs, 2.7 views
// per Gaussian on average, while some lane of a wavefront has one in 84 % of
// the wavefront-views), so the pairs are compacted before the expensive part:
//  1. scan: wavefront w reads, for its half of the views, every Gaussian's
//     gradient record and rectangle (all of them issued at once); the pairs
//     with a nonzero record over a nonempty rectangle go to its LDS list,
//     view by view;
//  2. rounds: the two lists, concatenated, are taken 64 pairs at a time by
//     the two wavefronts in turn; a lane takes one pair (the Gaussian's
//     parameters from its lane, its SH row and its view's camera from LDS)
//     and adds its contribution to the Gaussian's LDS accumulators with
//     double-precision LDS atomics (several views of one Gaussian may be
//     taken at once; the single-precision LDS atomic add measured several
//     times slower per instruction when most lanes take part);
//  3. wavefront 0 turns each Gaussian's sums into the raw-parameter
//     gradients, wavefront 1 copies the SH gradient out.
template <int DEG>
__global__ __launch_bounds__(128) void project_bwd_kernel(CamBatch cb, int64_t n, const float *__restrict__ means3d,
                                                         const float *__restrict__ log_scales,
                                                         const float *__restrict__ quats,
                                                         const float *__restrict__ logits,
                                                         const float *__restrict__ sh, const int4 *__restrict__ rect,
                                                         float *__restrict__ g_splats, bool clear,
                                                         float *__restrict__ d_means3d,
                                                         float *__restrict__ d_log_scales, float *__restrict__ d_quats,
                                                         float *__restrict__ d_logits, float *__restrict__ d_sh)
{
    constexpr int K3 = 3 * (DEG + 1) * (DEG + 1);
    constexpr int P = sh_stride(K3);
    constexpr int kHalf = kMaxViews / 2;
    __shared__ float s_sh[64 * P];
    __shared__ double s_dsh[K3 * kDshStride];    // coefficient-major: [k][Gaussian]
    __shared__ double s_acc[kRawGradD][64];
    __shared__ uint16_t s_items[2][64 * kHalf];   // lane | view << 8, one list per wavefront
    __shared__ int s_w[2];
    __shared__ Cam s_cam[kMaxViews];            // the cameras, read per lane by the pair's view
    const int lane = __lane_id();
    const int wid = threadIdx.x >> 6;
    {
        // (from the kernel argument once per workgroup: a lane's own view in
        // a round would otherwise be a vector load of it, waited for at once)
        constexpr int kCamWords = (int)(sizeof(Cam) / 4);
        static_assert(sizeof(Cam) % 4 == 0, "whole words");
        const int *src = reinterpret_cast<const int *>(cb.cam);
        int *dst = reinterpret_cast<int *>(s_cam);
        for (int e = threadIdx.x; e < cb.V * kCamWords; e += blockDim.x) dst[e] = src[e];
    }
    const int64_t g0 = (int64_t)blockIdx.x * 64;
    const int cnt = (int)min((int64_t)64, n - g0);
    if (wid == 0) {
        stage_sh<K3>(sh, g0, cnt, s_sh);
    } else {
        for (int k = 0; k < K3; ++k) s_dsh[k * kDshStride + lane] = 0.0;
        for (int c = 0; c < kRawGradD; ++c) s_acc[c][lane] = 0.0;
    }
    const bool in = lane < cnt;
    const int64_t i = g0 + (in ? lane : 0);
    const float m3[3] = {means3d[3 * i], means3d[3 * i + 1], means3d[3 * i + 2]};
    const float ls[3] = {log_scales[3 * i], log_scales[3 * i + 1], log_scales[3 * i + 2]};
    const float4 q4 = reinterpret_cast<const float4 *>(quats)[i];
    const float qt[4] = {q4.x, q4.y, q4.z, q4.w};
    const GaussPre G = gauss_pre(m3, ls, qt, logits[i]);

    // 1. scan: wavefront w takes views [w * h, min(V, (w + 1) * h)), h = ceil(V / 2)
    const int h = (cb.V + 1) >> 1;
    const int vbeg = wid * h, vend = min(cb.V, vbeg + h);
    int W = 0;
    {
        float gv[kHalf][kGradF];
        int4 rv[kHalf];
#pragma unroll
        for (int u = 0; u < kHalf; ++u) {
            const int64_t o = (int64_t)min(vbeg + u, cb.V - 1) * n + i;
            const float *gr = g_splats + (uint64_t)o * kGradF;
#pragma unroll
            for (int c = 0; c < kGradF; ++c) gv[u][c] = gr[c];
            rv[u] = rect[o];
        }
#pragma unroll
        for (int u = 0; u < kHalf; ++u) {
            const int v = vbeg + u;
            if (v >= vend) break;
            // a record that is not listed (nonzero over an empty rectangle:
            // nothing to add) is cleared here, a listed one when it is taken
            bool nz = false;
#pragma unroll
            for (int c = 0; c < kGradF; ++c) nz = nz || gv[u][c] != 0.f;
            nz = nz && in;
            const bool act = nz && rv[u].z > rv[u].x && rv[u].w > rv[u].y;
            if (clear && nz && !act) {
                float *gr = g_splats + ((uint64_t)v * n + i) * kGradF;
#pragma unroll
                for (int c = 0; c < kGradF; ++c) gr[c] = 0.f;
            }
            const uint64_t b = __ballot(act);
            const int pos = W + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32),
                                                              __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
            if (act) s_items[wid][pos] = (uint16_t)(lane | (v << 8));
            W += __popcll(b);
        }
    }
    if (lane == 0) s_w[wid] = W;
    __syncthreads();
    const int W0 = s_w[0], Wt = W0 + s_w[1];
    auto item = [&](int j) { return j < W0 ? (int)s_items[0][j] : (int)s_items[1][j - W0]; };

    // 2. rounds of 64 listed pairs, taken alternately by the two wavefronts
    float gn[kGradF];
    auto fetch = [&](int j) {
        if (j < Wt) {
            const int it = item(j);
            const float *gr = g_splats + ((uint64_t)(it >> 8) * n + (uint64_t)(g0 + (it & 63))) * kGradF;
#pragma unroll
            for (int c = 0; c < kGradF; ++c) gn[c] = gr[c];
        }
    };
    fetch(wid * 64 + lane);
    for (int r = wid * 64; r < Wt; r += 128) {
        const int j = r + lane;
        const bool has = j < Wt;
        const int it = has ? item(j) : 0;
        const int gl = it & 63, v = it >> 8;
        float gv[kGradF];
#pragma unroll
        for (int c = 0; c < kGradF; ++c) gv[c] = gn[c];
        fetch(j + 128);
        // the Gaussian's mean and view-independent terms, from its lane
        const int src4 = gl << 2;
        const float m3o[3] = {from_lane(m3[0], src4), from_lane(m3[1], src4), from_lane(m3[2], src4)};
        GaussPre Go;
        Go.ok = __builtin_amdgcn_ds_bpermute(src4, G.ok ? 1 : 0) != 0;
        for (int c = 0; c < 4; ++c) Go.qn[c] = from_lane(G.qn[c], src4);
        for (int c = 0; c < 3; ++c) Go.s[c] = from_lane(G.s[c], src4);
        Go.o = from_lane(G.o, src4);
        Go.qlen = 0.0;                          // unused by the per-view terms
        Go.tau = 0.0;
        if (has) {
            float *gr = g_splats + ((uint64_t)v * n + (uint64_t)(g0 + gl)) * kGradF;
            if (clear) {
#pragma unroll
                for (int c = 0; c < kGradF; ++c) gr[c] = 0.f;
            }
            const float gc3[3] = {gv[0], gv[1], gv[2]};
            const float gr3[3] = {gv[6], gv[7], gv[8]};
            RawGrad vg;
            if (project_bwd_view<DEG, double>(s_cam[v], m3o, Go, s_sh + gl * P, make_float2(gv[4], gv[5]), gc3, gv[3], gr3,
                                      vg, s_dsh + gl, kDshStride)) {
                for (int c = 0; c < 3; ++c) atomicAdd(&s_acc[c][gl], vg.m[c]);
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) atomicAdd(&s_acc[3 + 3 * a + b][gl], vg.M[a][b]);
                atomicAdd(&s_acc[12][gl], vg.logit);
            }
        }
    }
    __syncthreads();

    // 3. wavefront 0: the sums through the scales and the rotation; 1: the SH gradient
    if (wid == 0) {
        if (in) {
            double M[3][3];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) M[a][b] = s_acc[3 + 3 * a + b][lane];
            double gls[3] = {0.0, 0.0, 0.0}, gq[4] = {0.0, 0.0, 0.0, 0.0};
            if (G.ok) rot_scale_grad(G, M, gls, gq);
            for (int k = 0; k < 3; ++k) {
                d_means3d[3 * i + k] = (float)s_acc[k][lane];
                d_log_scales[3 * i + k] = (float)gls[k];
            }
            for (int k = 0; k < 4; ++k) d_quats[4 * i + k] = (float)gq[k];
            d_logits[i] = (float)s_acc[12][lane];
        }
    } else {
        unstage_dsh<K3>(d_sh, g0, cnt, s_dsh);
    }
}

}  // namespace
}  // namespace lgs

using namespace lgs;

static bool cams_from(const lgs_camera *cameras, int32_t V, CamBatch &cb)
{
    if (!cameras || V < 1 || V > kMaxViews) return false;
    cb.V = V;
    for (int v = 0; v < V; ++v)
        if (!cam_from(&cameras[v], cb.cam[v])) return false;
    for (int v = V; v < kMaxViews; ++v) cb.cam[v] = cb.cam[0];
    return true;
}

extern "C" lgs_status lgs_project_batch(const lgs_camera *cameras, int32_t num_views, int64_t n, int32_t sh_degree,
                                        const float *means3d, const float *log_scales, const float *quats,
                                        const float *opacity_logits, const float *sh, float *splats, float *depth,
                                        int32_t *rect, void *stream)
{
    CamBatch cb;
    LGS_REQUIRE(cams_from(cameras, num_views, cb), "lgs_project: invalid camera(s) or num_views not in 1..%d",
                kMaxViews);
    LGS_REQUIRE(n >= 0, "lgs_project: n < 0");
    LGS_REQUIRE(sh_degree >= 0 && sh_degree <= 3, "lgs_project: sh_degree must be 0..3");
    if (n == 0) return LGS_OK;
    LGS_REQUIRE(means3d && log_scales && quats && opacity_logits && sh, "lgs_project: null input");
    LGS_REQUIRE(splats && depth && rect, "lgs_project: null output");
    LGS_REQUIRE(((uintptr_t)splats % 16 == 0) && ((uintptr_t)rect % 16 == 0) && ((uintptr_t)sh % 16 == 0)
                    && ((uintptr_t)quats % 16 == 0),
                "lgs_project: splats/rect/sh/quats must be 16-byte aligned");
    hipStream_t s = as_stream(stream);
    const dim3 grid(grid_for(n, 256)), block(256);
    auto *rc = reinterpret_cast<int4 *>(rect);
#define LGS_PF(D)                                                                                                 \
    hipLaunchKernelGGL(project_fwd_kernel<D>, grid, block, 0, s, cb, n, means3d, log_scales, quats, opacity_logits, \
                       sh, splats, depth, rc)
    switch (sh_degree) {
    case 0: LGS_PF(0); break;
    case 1: LGS_PF(1); break;
    case 2: LGS_PF(2); break;
    default: LGS_PF(3); break;
    }
#undef LGS_PF
    LGS_LAUNCHED("lgs_project");
    return LGS_OK;
}

extern "C" lgs_status lgs_project(const lgs_camera *camera, int64_t n, int32_t sh_degree, const float *means3d,
                                  const float *log_scales, const float *quats, const float *opacity_logits,
                                  const float *sh, float *splats, float *depth, int32_t *rect, void *stream)
{
    return lgs_project_batch(camera, 1, n, sh_degree, means3d, log_scales, quats, opacity_logits, sh, splats, depth,
                             rect, stream);
}

extern "C" lgs_status lgs_project_backward_batch(const lgs_camera *cameras, int32_t num_views, int64_t n,
                                                 int32_t sh_degree, const float *means3d, const float *log_scales,
                                                 const float *quats, const float *opacity_logits, const float *sh,
                                                 const int32_t *rect, float *g_splats, float *d_means3d,
                                                 float *d_log_scales, float *d_quats, float *d_opacity_logits,
                                                 float *d_sh, int32_t flags, void *stream)
{
    CamBatch cb;
    LGS_REQUIRE(cams_from(cameras, num_views, cb),
                "lgs_project_backward: invalid camera(s) or num_views not in 1..%d", kMaxViews);
    LGS_REQUIRE(n >= 0, "lgs_project_backward: n < 0");
    LGS_REQUIRE(sh_degree >= 0 && sh_degree <= 3, "lgs_project_backward: sh_degree must be 0..3");
    LGS_REQUIRE((flags & ~LGS_PROJ_BWD_CLEAR) == 0, "lgs_project_backward: unknown flags %d", flags);
    if (n == 0) return LGS_OK;
    LGS_REQUIRE(means3d && log_scales && quats && opacity_logits && sh && rect, "lgs_project_backward: null input");
    LGS_REQUIRE(g_splats != nullptr, "lgs_project_backward: null gradient input");
    LGS_REQUIRE(d_means3d && d_log_scales && d_quats && d_opacity_logits && d_sh, "lgs_project_backward: null output");
    LGS_REQUIRE(((uintptr_t)g_splats % 4 == 0) && ((uintptr_t)rect % 16 == 0) && ((uintptr_t)sh % 16 == 0)
                    && ((uintptr_t)d_sh % 16 == 0) && ((uintptr_t)quats % 16 == 0),
                "lgs_project_backward: rect/sh/d_sh/quats must be 16-byte and g_splats 4-byte aligned");
    hipStream_t s = as_stream(stream);
    // up to kLoopViews views: one lane per Gaussian loops over them; more:
    // the (Gaussian, view) pairs with a gradient are listed and taken 64 at a
    // time (64 Gaussians per workgroup of 128 threads either way)
    const bool loop = num_views <= kLoopViews;
    const dim3 grid(grid_for(n, loop ? 128 : 64)), block(128);
    auto *rc = reinterpret_cast<const int4 *>(rect);
#define LGS_PB(D)                                                                                                   \
    hipLaunchKernelGGL(loop ? project_bwd_loop_kernel<D> : project_bwd_kernel<D>, grid, block, 0, s, cb, n, means3d,   \
                       log_scales, quats, opacity_logits, sh, rc, g_splats, (flags & LGS_PROJ_BWD_CLEAR) != 0,        \
                       d_means3d, d_log_scales, d_quats, d_opacity_logits, d_sh)
    switch (sh_degree) {
    case 0: LGS_PB(0); break;
    case 1: LGS_PB(1); break;
    case 2: LGS_PB(2); break;
    default: LGS_PB(3); break;
    }
#undef LGS_PB
    LGS_LAUNCHED("lgs_project_backward");
    return LGS_OK;
}

extern "C" lgs_status lgs_project_backward(const lgs_camera *camera, int64_t n, int32_t sh_degree,
                                           const float *means3d, const float *log_scales, const float *quats,
                                           const float *opacity_logits, const float *sh, const int32_t *rect,
                                           float *g_splats, float *d_means3d, float *d_log_scales,
                                           float *d_quats, float *d_opacity_logits, float *d_sh, int32_t flags,
                                           void *stream)
{
    return lgs_project_backward_batch(camera, 1, n, sh_degree, means3d, log_scales, quats, opacity_logits, sh, rect,
                                      g_splats, d_means3d, d_log_scales, d_quats,
                                      d_opacity_logits, d_sh, flags, stream);
}
