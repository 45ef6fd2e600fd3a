// Adaptation decisions of Sec. 4: Doerfler marking of the elements by their indicators and
// the smoothness sensor that chooses between p-enrichment and mesh refinement.
//
// Marking: the smallest set M of elements with eta_M >= (1 - theta) eta_T, where the error of
// a set is eta_M^2 = sum_{K in M} eta_K^2. Taking the elements in order of decreasing eta_K
// (ties by increasing element id: a stable sort) gives that set: M is the first m elements,
// m the first count whose partial sum of eta_K^2 reaches (1 - theta)^2 eta_T^2.
// Sensor: S_K = (w - w*, w - w*)_K / (w, w)_K with w* the projection onto the polynomials
// of degree p_K - 1; with the orthonormal hierarchical basis, w - w* is the part of the
// expansion in the modes of degree exactly p_K, and det J cancels:
//   S_K = sum_a sum_{deg(i) = p_K} W_a,i^2 / sum_a sum_{i < Np} W_a,i^2.
// A marked element with S_K < eps_S is flagged for p-enrichment (1), otherwise for mesh
// refinement (2); unmarked elements get 0.
#include <hipcub/hipcub.hpp>

#include <mutex>
#include <string>

#include "hdg_internal.h"

namespace hdg {

namespace {

constexpr int kScanThreads = 1024;

// Sensor and sort input of the elements of one bucket (degree p), one thread per element.
__global__ void k_sensor(const ElemInfo* einfo, int start, int count, int p, const double* w, int npmax,
                         const double* eta, double* sensor, double* key, int32_t* id) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const int e = einfo[start + t].elem;
    const int n0 = p * (p + 1) / 2, n1 = (p + 1) * (p + 2) / 2;   // modes of degree p: [n0, n1)
    double top = 0.0, all = 0.0;
    for (int a = 0; a < 4; ++a) {
        const double* wa = w + ((int64_t)e * 4 + a) * npmax;
        for (int i = 0; i < n1; ++i) {
            const double v = wa[i] * wa[i];
            all += v;
            if (i >= n0) top += v;
        }
    }
    sensor[e] = all > 0.0 ? top / all : 0.0;
    key[e] = eta[e];
    id[e] = e;
}

// Partial sums of eta^2 in sorted order, one workgroup: each thread sums a contiguous chunk in
// order, thread 0 accumulates the chunk totals in order, then each thread walks its chunk again
// from its base and records the first position whose partial sum reaches the target.
__global__ __launch_bounds__(kScanThreads) void k_dorfler(int n, const double* key_sorted, double theta,
                                                          int32_t* m_out) {
    __shared__ double base[kScanThreads + 1];
    __shared__ int first;
    const int t = threadIdx.x;
    const int chunk = (n + kScanThreads - 1) / kScanThreads;
    const int lo = min(n, t * chunk), hi = min(n, lo + chunk);
    double s = 0.0;
    for (int i = lo; i < hi; ++i) s += key_sorted[i] * key_sorted[i];
    base[t + 1] = s;
    if (t == 0) first = n;
    __syncthreads();
    if (t == 0) {
        base[0] = 0.0;
        for (int k = 1; k <= kScanThreads; ++k) base[k] += base[k - 1];
    }
    __syncthreads();
    const double target = (1.0 - theta) * (1.0 - theta) * base[kScanThreads];
    if (!(target > 0.0)) {
        if (t == 0) m_out[0] = 0;
        return;
    }
    double c = base[t];
    for (int i = lo; i < hi; ++i) {
        c += key_sorted[i] * key_sorted[i];
        if (c >= target) {
            atomicMin(&first, i);
            break;
        }
    }
    __syncthreads();
    if (t == 0) m_out[0] = first < n ? first + 1 : n;
}

__global__ void k_mark(int n, const int32_t* id_sorted, const int32_t* m, const double* sensor, double eps_s,
                       int32_t* flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int e = id_sorted[i];
    flag[e] = i < m[0] ? (sensor[e] < eps_s ? 1 : 2) : 0;
}

}  // namespace

int64_t mark_sort_temp_bytes(int n) {
    size_t bytes = 0;
    if (hipcub::DeviceRadixSort::SortPairsDescending(nullptr, bytes, (const double*)nullptr, (double*)nullptr,
                                                     (const int32_t*)nullptr, (int32_t*)nullptr, n) != hipSuccess)
        return -1;
    return (int64_t)bytes;
}

hipError_t launch_mark(const Plan& p, const double* w, const double* eta, double theta, double eps_s,
                       double* sensor, int32_t* flag, char* scratch, int32_t* m_dev, hipStream_t s) {
    const int n = p.ne;
    if (n == 0) return hipSuccess;
    double* key = (double*)scratch;
    double* key_sorted = key + n;
    int32_t* id = (int32_t*)(key_sorted + n);
    int32_t* id_sorted = id + n;
    void* temp = (void*)(((uintptr_t)(id_sorted + n) + 255) / 256 * 256);
    for (const Bucket& bk : p.buckets)
        hipLaunchKernelGGL(k_sensor, dim3((bk.count + 255) / 256), dim3(256), 0, s, p.d_einfo, bk.start, bk.count,
                           bk.p, w, p.npmax, eta, sensor, key, id);
    size_t bytes = (size_t)p.mark_temp_bytes;
    hipError_t e = hipcub::DeviceRadixSort::SortPairsDescending(temp, bytes, key, key_sorted, id, id_sorted, n, 0,
                                                                 64, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dorfler, dim3(1), dim3(kScanThreads), 0, s, n, key_sorted, theta, m_dev);
    hipLaunchKernelGGL(k_mark, dim3((n + 255) / 256), dim3(256), 0, s, n, id_sorted, m_dev, sensor, eps_s, flag);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Allocation-free marking: the same kernels on a scratch buffer that is a file-scope device
// array (one copy per GPU, held until the process ends) instead of the caller's workspace.
// Layout as in the workspace's marking region: the marked count (256 bytes), the sensor when
// the caller passes none (ne doubles), then the sort buffers and the radix-sort scratch.
// ---------------------------------------------------------------------------
constexpr int64_t kMarkScratchMax = (int64_t)16 << 20;   // 16 MiB per GPU

static __device__ __align__(256) char scratch[kMarkScratchMax];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
char* g_scratch_ptr[kMaxDevices] = {};   // device address of `scratch` on each GPU
}  // namespace

int64_t mark_noalloc_need(const Plan& p, bool own_sensor) {
    return 256 + (own_sensor ? (int64_t)p.ne * 8 : 0) + mark_scratch_bytes(p);
}

hdg_status mark_elements_noalloc(const Plan& p, const double* w, const double* eta, double theta, double eps_s,
                                 int32_t* flag, double* sensor, int32_t* n_marked_host, hipStream_t s) {
    const int64_t need = mark_noalloc_need(p, sensor == nullptr);
    if (need > kMarkScratchMax) {
        set_error("hdg_mark_elements_noalloc: the mesh needs " + std::to_string(need) +
                  " bytes of marking scratch, more than the static " + std::to_string(kMarkScratchMax) +
                  " (use hdg_mark_elements with a workspace)");
        return HDG_ERR_INVALID_ARG;
    }
    hipError_t e = hipSetDevice(p.device);
    if (e != hipSuccess || p.device < 0 || p.device >= kMaxDevices) {
        set_error(std::string("hdg_mark_elements_noalloc: device ") + std::to_string(p.device) + ": " +
                  hipGetErrorString(e));
        return e == hipSuccess ? HDG_ERR_INVALID_ARG : HDG_ERR_HIP;
    }
    char* base = nullptr;
    {
        // once per device, with that device current: the array's address on this GPU
        std::lock_guard<std::mutex> lock(g_scratch_mutex);
        if (!g_scratch_ptr[p.device]) {
            void* ptr = nullptr;
            e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr) {
                set_error(std::string("hdg_mark_elements_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
                return HDG_ERR_HIP;
            }
            g_scratch_ptr[p.device] = (char*)ptr;
        }
        base = g_scratch_ptr[p.device];
    }
    int32_t* m_dev = (int32_t*)base;
    double* sens = sensor ? sensor : (double*)(base + 256);
    char* sort = base + 256 + (sensor ? 0 : (int64_t)p.ne * 8);
    e = launch_mark(p, w, eta, theta, eps_s, sens, flag, sort, m_dev, s);
    if (e != hipSuccess) {
        set_error(std::string("hdg_mark_elements_noalloc: ") + hipGetErrorString(e));
        return HDG_ERR_HIP;
    }
    if (n_marked_host) {
        if (p.ne == 0) {
            *n_marked_host = 0;
            return HDG_OK;
        }
        e = hipMemcpyAsync(n_marked_host, m_dev, 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            set_error(std::string("hdg_mark_elements_noalloc: ") + hipGetErrorString(e));
            return HDG_ERR_HIP;
        }
    }
    return HDG_OK;
}

}  // namespace hdg
