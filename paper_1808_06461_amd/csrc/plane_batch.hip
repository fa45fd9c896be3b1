// Plane phase: batched launches of an ensemble.
#include "plane.hpp"

namespace chn {

template <typename T>
hipError_t launch_plane_batch(const BatchPlan<T>& b, hipStream_t st) {
  // the batched kernels take the classic radix passes (ensemble channels keep radix set 0)
  CHN_STAGED(T, b.mz, hipLaunchKernelGGL((k_zinv_batch<T, MV>), dim3(b.nz), dim3(256), b.lds_z, st, b.zinv, b.wz));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  CHN_ROWS(b.rz, CHN_STAGED(T, b.mx, hipLaunchKernelGGL((k_xpass_batch<T, MV, RZ>), dim3(b.nx), dim3(256), b.lds_x, st, b.xpass, b.wx)));
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  CHN_STAGED(T, b.mz, hipLaunchKernelGGL((k_zfwd_batch<T, MV>), dim3(b.nz), dim3(256), b.lds_z, st, b.zfwd, b.wz));
  return hipGetLastError();
}
template hipError_t launch_plane_batch<double>(const BatchPlan<double>&, hipStream_t);
template hipError_t launch_plane_batch<float>(const BatchPlan<float>&, hipStream_t);

}  // namespace chn
