// Instantiation of the decode kernels: double PCG vectors, hot arena in global memory.
#include "lpdec_kernels.hpp"

namespace lpdec {
LPDEC_INSTANTIATE(f64_glb, double, false)
}  // namespace lpdec
