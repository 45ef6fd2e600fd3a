// Kernels of the relaxed Newton iteration (Sec. 3.3): the residual norm ||N_h||_2 from the
// partials that the condensation kernels leave behind, and the update x <- x + dx.
//
// Residual rows: every element row of every element (Navier-Stokes: gradient and
// conserved-variable rows) and every skeleton row, the latter the sum of the two
// neighbours' shares. The condensation kernels write the squared norm of each element's
// rows (res_elem, one double per element) and each side's share of the skeleton rows
// (rl_part, the slots of the condensed right-hand side). The norm is reduced in a fixed
// order over a fixed grid, so repeated calls return the same bits.
#include <algorithm>

#include "hdg_internal.h"

namespace hdg {

namespace {

constexpr int kResThreads = 256;

__device__ __forceinline__ double block_sum_256(double v, double* red) {
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
#pragma unroll
    for (int s = kResThreads / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    return red[0];
}

// Thread i of the grid-stride sweep takes element i and face i.
__global__ __launch_bounds__(kResThreads) void k_res_partials(int ne, int nf, const double* res_elem,
                                                              const int64_t* face_off, const double* rl_part,
                                                              double* partials) {
    __shared__ double red[kResThreads];
    double s = 0.0;
    const int n = ne > nf ? ne : nf;
    for (int i = blockIdx.x * kResThreads + threadIdx.x; i < n; i += gridDim.x * kResThreads) {
        if (i < ne) s += res_elem[i];
        if (i < nf) {
            const int64_t o = face_off[i], se = face_off[i + 1] - o;
            const double* g = rl_part + 2 * o;
            for (int64_t t = 0; t < se; ++t) {
                const double v = g[t] + g[se + t];
                s += v * v;
            }
        }
    }
    const double b = block_sum_256(s, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = b;
}

__global__ __launch_bounds__(kResThreads) void k_res_final(int nb, const double* partials, double* out) {
    __shared__ double red[kResThreads];
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += kResThreads) s += partials[i];
    const double b = block_sum_256(s, red);
    if (threadIdx.x == 0) out[0] = sqrt(b);
}

__global__ __launch_bounds__(256) void k_axpy_update(int64_t n, double* x, const double* dx) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) x[i] += dx[i];
}

}  // namespace

hipError_t launch_residual_norm(const Plan& p, const double* res_elem, const double* rl_part, double* partials,
                                double* out_dev, hipStream_t s) {
    const int n = std::max(p.ne, p.nf);
    int nb = (n + kResThreads - 1) / kResThreads;
    nb = std::max(1, std::min(nb, kResPartials));
    hipLaunchKernelGGL(k_res_partials, dim3(nb), dim3(kResThreads), 0, s, p.ne, p.nf, res_elem, p.d_face_off,
                       rl_part, partials);
    hipLaunchKernelGGL(k_res_final, dim3(1), dim3(kResThreads), 0, s, nb, partials, out_dev);
    return hipGetLastError();
}

hipError_t launch_axpy_update(int64_t n, double* x, const double* dx, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_axpy_update, dim3((unsigned)nb), dim3(256), 0, s, n, x, dx);
    return hipGetLastError();
}

}  // namespace hdg
