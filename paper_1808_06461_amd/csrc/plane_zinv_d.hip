// Plane phase: z inverse launcher, float64 transforms.
#include "plane.hpp"

namespace chn {

template <typename T>
hipError_t launch_zinv(const ZinvArgs<T>& a, hipStream_t st) {
  dim3 grid((a.d.n1h + a.K - 1) / a.K, a.ny);
  size_t sh = (size_t)a.K * a.lstride * sizeof(c2<T>);
  if (z_threads(a.plan, a.K) == 1024) {
    // runtime schedule: the compile-time 9216-point one spills at 1024 threads
    // (128 VGPRs) and is slower here; the forward pass below keeps it
    const int m = pick_staging<T>(a.plan, 1, 1024);
    if (plan_is_composite(a.plan))
      CHN_STAGED(T, m, hipLaunchKernelGGL((k_zinv<T, MV, kFnComposite, 1024>), grid, dim3(1024), sh, st, a));
    else
      CHN_STAGED(T, m, hipLaunchKernelGGL((k_zinv<T, MV, 0, 1024>), grid, dim3(1024), sh, st, a));
    return hipGetLastError();
  }
  const int m = pick_staging<T>(a.plan, a.K, 256);
  const bool fx = a.fixed && plan_is_576(a.plan), cp = plan_is_composite(a.plan);
  const bool fc = a.fixed && plan_is_576c(a.plan);
  if (a.pipe) {
    if (fx) CHN_STAGED(T, m, hipLaunchKernelGGL((k_zinv<T, MV, 576, 256, true>), grid, dim3(256), sh, st, a));
    else if (fc) CHN_STAGED(T, m, hipLaunchKernelGGL((k_zinv<T, MV, kFn576Composite, 256, true>), grid, dim3(256), sh, st, a));
    else if (cp) CHN_STAGED(T, m, hipLaunchKernelGGL((k_zinv<T, MV, kFnComposite, 256, true>), grid, dim3(256), sh, st, a));
    else CHN_STAGED(T, m, hipLaunchKernelGGL((k_zinv<T, MV, 0, 256, true>), grid, dim3(256), sh, st, a));
  } else {
    if (fx) CHN_STAGED(T, m, hipLaunchKernelGGL((k_zinv<T, MV, 576>), grid, dim3(256), sh, st, a));
    else if (fc) CHN_STAGED(T, m, hipLaunchKernelGGL((k_zinv<T, MV, kFn576Composite>), grid, dim3(256), sh, st, a));
    else if (cp) CHN_STAGED(T, m, hipLaunchKernelGGL((k_zinv<T, MV, kFnComposite>), grid, dim3(256), sh, st, a));
    else CHN_STAGED(T, m, hipLaunchKernelGGL((k_zinv<T, MV, 0>), grid, dim3(256), sh, st, a));
  }
  return hipGetLastError();
}

template hipError_t launch_zinv<double>(const ZinvArgs<double>&, hipStream_t);

}  // namespace chn
