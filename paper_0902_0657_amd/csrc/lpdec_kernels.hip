// Host launchers of the decode kernels (the kernels themselves are instantiated in
// lpdec_inst_*.hip), the frame-ordering kernels of a batch, and the fixed device region of
// the allocation-free entry point.
#include <hip/hip_runtime.h>

#include <mutex>

#include "lpdec_device.hpp"
#include "lpdec_launch.hpp"

namespace lpdec {

size_t static_lds_bytes() { return sizeof(Scratch); }

// ---------------------------------------------------------------- dispatch order of a batch
// A launch lasts as long as its slowest workgroup chain: a hard frame whose workgroup is
// dispatched only after the first wave of frames has finished extends it. The decode therefore
// takes the frames by descending syndrome weight of their hard decisions (the number of checks
// the channel decisions violate), which tracks the number of cuts and LPs a frame needs. The
// order decides only which workgroup decodes a frame and when; every frame's result is the same.

__global__ void __launch_bounds__(256) order_clear(int32_t *hist, int nbins)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nbins) hist[i] = 0;
}

// one wave per frame: syndrome weight (lanes take checks in turn) and its histogram
__global__ void __launch_bounds__(64) order_weights(Args a, int32_t *w, int32_t *hist)
{
    const int f = blockIdx.x, lane = threadIdx.x;
    const CodeView &cd = a.code;
    const size_t off = (size_t)f * cd.n;
    int wt = 0;
    for (int j = lane; j < cd.m; j += 64) {
        int par = 0;
        for (int e = cd.rowptr[j]; e < cd.rowptr[j + 1]; ++e) {
            const size_t k = off + cd.col[e];
            const double g = a.gamma_f64 ? ((const double *)a.gamma)[k] : (double)((const float *)a.gamma)[k];
            par ^= g < 0.0 ? 1 : 0;
        }
        wt += par;
    }
    for (int d = 32; d > 0; d >>= 1) wt += __shfl_xor(wt, d, 64);
    if (lane == 0) {
        w[f] = wt;
        atomicAdd(&hist[wt], 1);
    }
}

// one workgroup: hist[v] becomes the number of frames of weight above v (the first position of
// weight v in the order)
__global__ void __launch_bounds__(256) order_bases(int32_t *hist, int nbins)
{
    __shared__ int part[256];
    const int t = threadIdx.x, nt = blockDim.x;
    const int chunk = (nbins + nt - 1) / nt;
    // thread t owns bins top - t*chunk down to top - (t+1)*chunk + 1 (descending weights)
    const int hi = nbins - 1 - t * chunk, lo = max(hi - chunk + 1, 0);
    int sum = 0;
    for (int v = hi; v >= lo; --v) sum += hist[v];
    part[t] = sum;
    __syncthreads();
    if (t == 0) {
        int run = 0;
        for (int k = 0; k < nt; ++k) {
            const int c = part[k];
            part[k] = run;
            run += c;
        }
    }
    __syncthreads();
    int run = part[t];
    for (int v = hi; v >= lo; --v) {
        const int c = hist[v];
        hist[v] = run;
        run += c;
    }
}

// one workgroup: each frame's position, frames of equal weight in index order. Chunks of 256
// frames in turn; a frame's rank among the equal-weight frames before it in the chunk is counted
// in LDS, and the chunk's last frame of each weight advances that weight's next position.
__global__ void __launch_bounds__(256) order_scatter(int nframes, const int32_t *w, int32_t *hist, int32_t *order)
{
    __shared__ int wl[256];
    const int t = threadIdx.x;
    for (int c0 = 0; c0 < nframes; c0 += 256) {
        const int f = c0 + t;
        const int wf = f < nframes ? w[f] : -1;
        wl[t] = wf;
        __syncthreads();
        int rank = 0;
        bool last = true;
        if (wf >= 0) {
            for (int k = 0; k < t; ++k) rank += wl[k] == wf ? 1 : 0;
            for (int k = t + 1; k < 256; ++k)
                if (wl[k] == wf) { last = false; break; }
            order[hist[wf] + rank] = f;
        }
        __syncthreads();   // every frame of the chunk has read its weight's position
        if (wf >= 0 && last) hist[wf] += rank + 1;
        __syncthreads();
    }
}

hipError_t launch_order(const Args &a, int32_t *order, int32_t *w, int32_t *hist, hipStream_t stream)
{
    (void)hipGetLastError();
    const int nbins = a.code.m + 1;
    const int gb = (nbins + 255) / 256;
    hipLaunchKernelGGL(order_clear, dim3(gb), dim3(256), 0, stream, hist, nbins);
    hipLaunchKernelGGL(order_weights, dim3(a.nframes), dim3(64), 0, stream, a, w, hist);
    hipLaunchKernelGGL(order_bases, dim3(1), dim3(256), 0, stream, hist, nbins);
    hipLaunchKernelGGL(order_scatter, dim3(1), dim3(256), 0, stream, a.nframes, (const int32_t *)w, hist, order);
    return hipGetLastError();
}

hipError_t launch_main(const Args &a, int pt64, int block, size_t lds_bytes, hipStream_t stream, int grid)
{
    if (pt64) return a.hot_in_lds ? launch_f64_lds(a, block, lds_bytes, stream, grid)
                                  : launch_f64_glb(a, block, lds_bytes, stream, grid);
    return a.hot_in_lds ? launch_f32_lds(a, block, lds_bytes, stream, grid)
                        : launch_f32_glb(a, block, lds_bytes, stream, grid);
}

int decode_per_cu(int pt64, int hot_in_lds, int block, size_t lds_bytes)
{
    const void *fn = pt64 ? (hot_in_lds ? decode_kernel_f64_lds() : decode_kernel_f64_glb())
                          : (hot_in_lds ? decode_kernel_f32_lds() : decode_kernel_f32_glb());
    if (lds_bytes > 0)
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, block, lds_bytes) != hipSuccess || nb < 1) nb = 1;
    (void)hipGetLastError();
    return nb;
}

// Workspace of lpdec_decode_batch_noalloc: a fixed region of device memory that every call on
// a device shares (each device holds its own copy from the load of the library's code object
// until the process ends). Host code must not pass the symbol itself to a kernel: its name
// there is a host-side stand-in, not a device address. scratch_region looks the device address
// up once per device and hands out that address only.
static __device__ __align__(256) char scratch[kScratchBytes];

hipError_t scratch_region(int device, char **ptr)
{
    static std::mutex mu;
    static char *addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        char *p = nullptr;
        // the caller has made `device` current
        const hipError_t e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = p;
    }
    *ptr = addr[device];
    return hipSuccess;
}

hipError_t launch_clear(int32_t *p, int n, hipStream_t stream)
{
    (void)hipGetLastError();
    hipLaunchKernelGGL(order_clear, dim3((n + 255) / 256), dim3(256), 0, stream, p, n);
    return hipGetLastError();
}

}  // namespace lpdec
