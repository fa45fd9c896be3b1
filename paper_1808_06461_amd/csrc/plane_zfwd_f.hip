// Plane phase: z forward launcher, float32 transforms.
#include "plane.hpp"

namespace chn {

template <typename T, typename TO>
hipError_t launch_zfwd(const ZfwdArgs<T, TO>& a, hipStream_t st) {
  dim3 grid((a.d.n1h + a.K - 1) / a.K, a.ny);
  size_t sh = (size_t)a.K * a.lstride * sizeof(c2<T>);
  if (z_threads(a.plan, a.K) == 1024) {
    const int m = pick_staging<T>(a.plan, 1, 1024);
    if (a.fixed && plan_is_9216(a.plan))
      CHN_STAGED(T, m, hipLaunchKernelGGL((k_zfwd<T, TO, MV, 9216, 1024>), grid, dim3(1024), sh, st, a));
    else if (plan_is_composite(a.plan))
      CHN_STAGED(T, m, hipLaunchKernelGGL((k_zfwd<T, TO, MV, kFnComposite, 1024>), grid, dim3(1024), sh, st, a));
    else
      CHN_STAGED(T, m, hipLaunchKernelGGL((k_zfwd<T, TO, MV, 0, 1024>), grid, dim3(1024), sh, st, a));
    return hipGetLastError();
  }
  const int m = pick_staging<T>(a.plan, a.K, 256);
  const bool fx = a.fixed && plan_is_576(a.plan), cp = plan_is_composite(a.plan);
  const bool fc = a.fixed && plan_is_576c(a.plan);
  if (a.pipe) {
    if (fx) CHN_STAGED(T, m, hipLaunchKernelGGL((k_zfwd<T, TO, MV, 576, 256, true>), grid, dim3(256), sh, st, a));
    else if (fc) CHN_STAGED(T, m, hipLaunchKernelGGL((k_zfwd<T, TO, MV, kFn576Composite, 256, true>), grid, dim3(256), sh, st, a));
    else if (cp) CHN_STAGED(T, m, hipLaunchKernelGGL((k_zfwd<T, TO, MV, kFnComposite, 256, true>), grid, dim3(256), sh, st, a));
    else CHN_STAGED(T, m, hipLaunchKernelGGL((k_zfwd<T, TO, MV, 0, 256, true>), grid, dim3(256), sh, st, a));
  } else {
    if (fx) CHN_STAGED(T, m, hipLaunchKernelGGL((k_zfwd<T, TO, MV, 576>), grid, dim3(256), sh, st, a));
    else if (fc) CHN_STAGED(T, m, hipLaunchKernelGGL((k_zfwd<T, TO, MV, kFn576Composite>), grid, dim3(256), sh, st, a));
    else if (cp) CHN_STAGED(T, m, hipLaunchKernelGGL((k_zfwd<T, TO, MV, kFnComposite>), grid, dim3(256), sh, st, a));
    else CHN_STAGED(T, m, hipLaunchKernelGGL((k_zfwd<T, TO, MV, 0>), grid, dim3(256), sh, st, a));
  }
  return hipGetLastError();
}

template hipError_t launch_zfwd<float, float>(const ZfwdArgs<float, float>&, hipStream_t);
template hipError_t launch_zfwd<float, double>(const ZfwdArgs<float, double>&, hipStream_t);

}  // namespace chn
