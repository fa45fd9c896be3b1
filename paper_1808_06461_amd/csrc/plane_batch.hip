// Plane phase: batched launches of an ensemble.
#include "plane.hpp"

namespace chn {

template <typename T, int FN, int FX>
hipError_t launch_plane_batch_fn(const BatchPlan<T>& b, hipStream_t st) {
  CHN_STAGED(T, b.mz, hipLaunchKernelGGL((k_zinv_batch<T, MV, FN>), dim3(b.nz), dim3(256), b.lds_z, st, b.zinv, b.wz));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  CHN_ROWS(b.rz, CHN_STAGED(T, b.mx, hipLaunchKernelGGL((k_xpass_batch<T, MV, RZ, FX>), dim3(b.nx), dim3(256), b.lds_x, st, b.xpass, b.wx)));
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  CHN_STAGED(T, b.mz, hipLaunchKernelGGL((k_zfwd_batch<T, MV, FN>), dim3(b.nz), dim3(256), b.lds_z, st, b.zfwd, b.wz));
  return hipGetLastError();
}

// The composite form of the kernels takes plans of either radix set (the x
// pass's short lines of minimal channels on compile-time schedules; the z
// passes keep the runtime ones, which need fewer registers there).
template <typename T>
hipError_t launch_plane_batch(const BatchPlan<T>& b, hipStream_t st) {
  return b.comp ? launch_plane_batch_fn<T, kFnComposite, kFnShort>(b, st) : launch_plane_batch_fn<T, 0, 0>(b, st);
}
template hipError_t launch_plane_batch<double>(const BatchPlan<double>&, hipStream_t);
template hipError_t launch_plane_batch<float>(const BatchPlan<float>&, hipStream_t);

}  // namespace chn
