// Library-wide entry points: error reporting, version, L1 loss.
#include "common.hpp"

namespace lgs {

static thread_local char g_error[512] = "";

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_error, sizeof g_error, fmt, ap);
    va_end(ap);
}

lgs_status launch_status(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("%s: kernel launch failed: %s", what, hipGetErrorString(e));
        return LGS_ERR_HIP;
    }
    return LGS_OK;
}

namespace {

// L = mean |x - y|, dL/dx = sign(x - y) / count.  Each block writes its
// partial sum of |x - y| (double) to its own slot; one workgroup then adds the
// slots in a fixed order, so the loss is deterministic and a call touches no
// memory but its own arguments.
__global__ __launch_bounds__(256) void l1_kernel(const float *__restrict__ x, const float *__restrict__ y, int64_t n,
                                                 float inv_n, float *__restrict__ grad, double *__restrict__ partial)
{
    __shared__ double s_w[4];
    double sum = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float d = x[i] - y[i];
        grad[i] = d > 0.f ? inv_n : (d < 0.f ? -inv_n : 0.f);
        sum += fabs((double)d);
    }
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
    if (__lane_id() == 0) s_w[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (s_w[0] + s_w[1]) + (s_w[2] + s_w[3]);
}

__global__ __launch_bounds__(256) void l1_finish_kernel(const double *__restrict__ partial, int nparts,
                                                        float *__restrict__ loss, double inv_n)
{
    __shared__ double s_w[4];
    double sum = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 256) sum += partial[i];
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
    if (__lane_id() == 0) s_w[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) *loss = (float)(((s_w[0] + s_w[1]) + (s_w[2] + s_w[3])) * inv_n);
}

}  // namespace

lgs_status l1_launch(const float *image, const float *target, int64_t count, float *loss, float *grad,
                     double *partial, hipStream_t s)
{
    unsigned g = grid_for(count, 256);
    if (g > (unsigned)kL1Parts) g = kL1Parts;
    hipLaunchKernelGGL(l1_kernel, dim3(g), dim3(256), 0, s, image, target, count, (float)(1.0 / (double)count), grad,
                       partial);
    hipLaunchKernelGGL(l1_finish_kernel, dim3(1), dim3(256), 0, s, (const double *)partial, (int)g, loss,
                       1.0 / (double)count);
    return launch_status("lgs_l1_loss");
}

}  // namespace lgs

using namespace lgs;

extern "C" const char *lgs_last_error(void) { return g_error; }

extern "C" const char *lgs_version(void) { return "localgs-gfx950 0.1"; }

extern "C" size_t lgs_l1_workspace_size(void) { return kL1Parts * sizeof(double); }

extern "C" lgs_status lgs_l1_loss(const float *image, const float *target, int64_t count, float *loss, float *grad,
                                  void *workspace, size_t workspace_bytes, void *stream)
{
    LGS_REQUIRE(count > 0 && image && target && loss && grad, "lgs_l1_loss: bad arguments");
    LGS_REQUIRE(workspace && workspace_bytes >= lgs_l1_workspace_size() && (uintptr_t)workspace % 8 == 0,
                "lgs_l1_loss: workspace must be 8-byte aligned and hold lgs_l1_workspace_size() bytes");
    return l1_launch(image, target, count, loss, grad, static_cast<double *>(workspace), as_stream(stream));
}
