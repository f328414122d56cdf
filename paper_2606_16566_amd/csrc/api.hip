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

// L = mean |x - y|, dL/dx = sign(x - y) / count.  Block partial sums are
// reduced in double and added with one atomic per block.
__global__ __launch_bounds__(256) void l1_kernel(const float *__restrict__ x, const float *__restrict__ y, int64_t n,
                                                 float inv_n, float *__restrict__ grad, double *__restrict__ acc)
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
    if (threadIdx.x == 0) atomicAdd(acc, s_w[0] + s_w[1] + s_w[2] + s_w[3]);
}

__global__ void l1_finish_kernel(double *acc, float *loss, double inv_n)
{
    *loss = (float)(*acc * inv_n);
    *acc = 0.0;
}

// one double accumulator per device for the loss reduction (cleared by
// l1_finish_kernel after every use, so it is zero between calls)
__device__ double g_l1_acc = 0.0;

}  // namespace
}  // namespace lgs

using namespace lgs;

extern "C" const char *lgs_last_error(void) { return g_error; }

extern "C" const char *lgs_version(void) { return "localgs-gfx950 0.1"; }

extern "C" lgs_status lgs_l1_loss(const float *image, const float *target, int64_t count, float *loss, float *grad,
                                  void *stream)
{
    LGS_REQUIRE(count > 0 && image && target && loss && grad, "lgs_l1_loss: bad arguments");
    hipStream_t s = as_stream(stream);
    // the accumulator's device address, looked up once per device (so the
    // call stays capturable into a graph)
    static double *acc_of[64] = {nullptr};
    int dev = 0;
    LGS_HIP(hipGetDevice(&dev));
    LGS_REQUIRE(dev >= 0 && dev < 64, "lgs_l1_loss: device index %d out of range", dev);
    if (!acc_of[dev]) LGS_HIP(hipGetSymbolAddress((void **)&acc_of[dev], HIP_SYMBOL(g_l1_acc)));
    double *acc = acc_of[dev];
    unsigned g = grid_for(count, 256);
    if (g > 2048) g = 2048;
    hipLaunchKernelGGL(l1_kernel, dim3(g), dim3(256), 0, s, image, target, count, (float)(1.0 / (double)count), grad,
                       acc);
    hipLaunchKernelGGL(l1_finish_kernel, dim3(1), dim3(1), 0, s, acc, loss, 1.0 / (double)count);
    LGS_LAUNCHED("lgs_l1_loss");
    return LGS_OK;
}
