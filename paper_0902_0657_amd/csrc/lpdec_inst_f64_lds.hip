// Instantiation of the decode kernels: double PCG vectors, hot arena in LDS.
#include "lpdec_kernels.hpp"

namespace lpdec {
LPDEC_INSTANTIATE(f64_lds, double, true)
}  // namespace lpdec
