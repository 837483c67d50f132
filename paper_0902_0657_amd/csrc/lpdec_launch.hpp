// Host-side launcher of the per-frame decode kernel.
#pragma once
#include <hip/hip_runtime.h>

#include "lpdec_common.hpp"

namespace lpdec {

// The four instantiations of the decode kernels (lpdec_inst_*.hip): launchers for every mode,
// and the address of the MODE_DECODE kernel (for occupancy queries).
hipError_t launch_f64_lds(const Args &a, int block, size_t lds, hipStream_t s, int grid);
hipError_t launch_f64_glb(const Args &a, int block, size_t lds, hipStream_t s, int grid);
hipError_t launch_f32_lds(const Args &a, int block, size_t lds, hipStream_t s, int grid);
hipError_t launch_f32_glb(const Args &a, int block, size_t lds, hipStream_t s, int grid);
const void *decode_kernel_f64_lds();
const void *decode_kernel_f64_glb();
const void *decode_kernel_f32_lds();
const void *decode_kernel_f32_glb();
// Launches one workgroup per frame. pt64: PCG in FP64 (1) or FP32 (0). lds_bytes: dynamic
// LDS for the hot arena when a.hot_in_lds.
hipError_t launch_main(const Args &a, int pt64, int block, size_t lds_bytes, hipStream_t stream, int grid);
// Workgroups of the decode kernel (MODE_DECODE) that one compute unit holds at once.
int decode_per_cu(int pt64, int hot_in_lds, int block, size_t lds_bytes);
// Zeroes n ints on `stream` with a kernel (no memset node when the stream is captured).
hipError_t launch_clear(int32_t *p, int n, hipStream_t stream);
// Size of the fixed device region behind lpdec_decode_batch_noalloc, and the devices it is
// looked up for.
constexpr size_t kScratchBytes = (size_t)LPDEC_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
// Device address of that region on `device` (which must be current); looked up with
// hipGetSymbolAddress on the first call per device.
hipError_t scratch_region(int device, char **ptr);
// Static LDS used by the kernel besides the hot arena.
size_t static_lds_bytes();
// Dispatch order of a decode batch (a.nframes frames of a.gamma): order[0..nframes) lists the
// frames by descending syndrome weight of their hard decisions. w holds nframes and hist
// m + 1 ints of scratch.
hipError_t launch_order(const Args &a, int32_t *order, int32_t *w, int32_t *hist, hipStream_t stream);

}  // namespace lpdec
