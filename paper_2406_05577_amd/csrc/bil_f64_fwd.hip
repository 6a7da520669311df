// Band-inner register-line kernels: double forward instantiations.
#include "kernels_bil.hpp"

namespace fftb {
FFTB_BIL_DECL(, -1, double)
}  // namespace fftb
