// Instantiation of the decode kernels: float PCG vectors, hot arena in global memory.
#include "lpdec_kernels.hpp"

namespace lpdec {
LPDEC_INSTANTIATE(f32_glb, float, false)
}  // namespace lpdec
