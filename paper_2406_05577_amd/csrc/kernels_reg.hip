// Register-path dispatch: shape tables and the launchers the host calls. The
// kernels themselves are templates in kernels_reg.hpp, instantiated in the
// reg_*.hip translation units.
#include "kernels_bil.hpp"

namespace fftb {

FFTB_REG_DECL_ALL(extern)
FFTB_BIL_DECL(extern, +1, float)
FFTB_BIL_DECL(extern, -1, float)
FFTB_BIL_DECL(extern, +1, double)
FFTB_BIL_DECL(extern, -1, double)

// Band-inner shapes: z lines (column kernel) or x lines (plane kernel); the
// narrow x lines (half a piece of bands per row) of the complex64 inverse
// plane kernel.
bool bil_shape_supported(bool fp64, bool zaxis, int E, int H) {
#define FFTB_CHK(e, h) if (E == e && H == h) return true;
  if (fp64) {
    if (zaxis) { FFTB_BIL_Z_F64(FFTB_CHK) } else { FFTB_BIL_X_F64(FFTB_CHK) }
  } else {
    if (zaxis) { FFTB_BIL_Z_F32(FFTB_CHK) } else { FFTB_BIL_X_F32(FFTB_CHK) }
  }
#undef FFTB_CHK
  return false;
}
bool bil_narrow_supported(bool fp64, int E, int H) {
  if (fp64) return false;
#define FFTB_CHK(e, h) if (E == e && H == h) return true;
  FFTB_BIL_XN_F32(FFTB_CHK)
#undef FFTB_CHK
  return false;
}

// which: 1 = column kernel (E, H of the z axis), 2 = plane kernel (E, H of x)
hipError_t launch_bil(int which, const KArgs& a, bool inverse, bool fp64, int E, int H, int grid,
                      int threads, size_t lds, hipStream_t st, int fold_m) {
  if (fp64)
    return inverse ? bil_dispatch<+1, double>(which, a, E, H, grid, threads, lds, st, fold_m, false)
                   : bil_dispatch<-1, double>(which, a, E, H, grid, threads, lds, st, fold_m, false);
  return inverse ? bil_dispatch<+1, float>(which, a, E, H, grid, threads, lds, st, fold_m, false)
                 : bil_dispatch<-1, float>(which, a, E, H, grid, threads, lds, st, fold_m, false);
}

// Allow the band-inner plane kernels of an x shape `lds` bytes of dynamic LDS
// (narrow: the narrow inverse kernels).
hipError_t prepare_bil(bool fp64, int E, int H, size_t lds, bool narrow) {
  KArgs dummy{};
  hipError_t e;
  if (narrow)
    return fp64 ? bil_dispatch<+1, double>(3, dummy, E, H, 0, 0, lds, nullptr, 0, true)
                : bil_dispatch<+1, float>(3, dummy, E, H, 0, 0, lds, nullptr, 0, true);
  if (fp64) {
    e = bil_dispatch<+1, double>(2, dummy, E, H, 0, 0, lds, nullptr, 0, true);
    return e != hipSuccess ? e : bil_dispatch<-1, double>(2, dummy, E, H, 0, 0, lds, nullptr, 0, true);
  }
  e = bil_dispatch<+1, float>(2, dummy, E, H, 0, 0, lds, nullptr, 0, true);
  return e != hipSuccess ? e : bil_dispatch<-1, float>(2, dummy, E, H, 0, 0, lds, nullptr, 0, true);
}

hipError_t launch_combine(const KArgs& a, bool fp64, int grid, int threads, hipStream_t st) {
  if (fp64)
    hipLaunchKernelGGL((k3r_kernel<double>), dim3(grid), dim3(threads), 0, st, a);
  else
    hipLaunchKernelGGL((k3r_kernel<float>), dim3(grid), dim3(threads), 0, st, a);
  return hipGetLastError();
}

bool reg_shape_supported(bool fp64, int E, int H) {
  (void)fp64;  // both precisions compile the same shapes
#define FFTB_CHK(e, h, p) if (E == e && H == h) return true;
  FFTB_REG_SHAPES(FFTB_CHK)
#undef FFTB_CHK
  return false;
}

bool mfma_shape_supported(bool fp64, int E, int H) { return !fp64 && E == 16 && H == 8; }

bool fold_m_supported(int H, int m) { return fold_m_compiled(H, m); }

namespace {
template <int S, typename T>
hipError_t dispatch_parts(int which, const KArgs& a, int E, int H, int grid, int threads,
                          size_t lds, hipStream_t st, int fold_m, bool attr_only) {
  bool found = false;
  hipError_t e = reg_dispatch<S, T, 0>(which, a, E, H, grid, threads, lds, st, fold_m, attr_only, &found);
  if (found) return e;
  e = reg_dispatch<S, T, 1>(which, a, E, H, grid, threads, lds, st, fold_m, attr_only, &found);
  if (found) return e;
  e = reg_dispatch<S, T, 2>(which, a, E, H, grid, threads, lds, st, fold_m, attr_only, &found);
  if (found) return e;
  return hipErrorInvalidValue;
}
}  // namespace

// which: 1 = column kernel (E, H of the z axis), 2 = plane kernel (E, H of x)
hipError_t launch_reg(int which, const KArgs& a, bool inverse, bool fp64, int E, int H, int grid,
                      int threads, size_t lds, hipStream_t st, bool mfma, int fold_m) {
  if (mfma) {
    if (fp64 || E != 16 || H != 8) return hipErrorInvalidValue;
    return inverse ? reg_dispatch_mfma<+1>(which, a, grid, threads, lds, st, fold_m, false)
                   : reg_dispatch_mfma<-1>(which, a, grid, threads, lds, st, fold_m, false);
  }
  if (fp64)
    return inverse ? dispatch_parts<+1, double>(which, a, E, H, grid, threads, lds, st, fold_m, false)
                   : dispatch_parts<-1, double>(which, a, E, H, grid, threads, lds, st, fold_m, false);
  return inverse ? dispatch_parts<+1, float>(which, a, E, H, grid, threads, lds, st, fold_m, false)
                 : dispatch_parts<-1, float>(which, a, E, H, grid, threads, lds, st, fold_m, false);
}

hipError_t prepare_reg(bool fp64, int E, int H, size_t lds, bool mfma) {
  KArgs dummy{};
  if (mfma) {
    if (fp64 || E != 16 || H != 8) return hipErrorInvalidValue;
    hipError_t err = reg_dispatch_mfma<+1>(2, dummy, 0, 0, lds, nullptr, 0, true);
    return err != hipSuccess ? err : reg_dispatch_mfma<-1>(2, dummy, 0, 0, lds, nullptr, 0, true);
  }
  hipError_t err;
  if (fp64) {
    err = dispatch_parts<+1, double>(2, dummy, E, H, 0, 0, lds, nullptr, 0, true);
    return err != hipSuccess ? err : dispatch_parts<-1, double>(2, dummy, E, H, 0, 0, lds, nullptr, 0, true);
  }
  err = dispatch_parts<+1, float>(2, dummy, E, H, 0, 0, lds, nullptr, 0, true);
  return err != hipSuccess ? err : dispatch_parts<-1, float>(2, dummy, E, H, 0, 0, lds, nullptr, 0, true);
}

}  // namespace fftb
