// Register-path kernels: F64 forward, shape part 0.
#include "kernels_reg.hpp"

namespace fftb {
template hipError_t reg_dispatch<-1, double, 0>(int, const KArgs&, int, int, int, int, size_t,
                                              hipStream_t, int, bool, bool*);
}  // namespace fftb
