// Plane phase: x pass launcher, float32 transforms.
#include "plane.hpp"

namespace chn {

template <typename T>
hipError_t launch_xpass(const XpassArgs<T>& a, hipStream_t st) {
  if (a.rows >= 2) {
    const int m = pick_staging<T>(a.plan, 3 * a.rows, 256);
    dim3 grid((a.d.p3 + a.rows - 1) / a.rows, a.ny);
    size_t sh = (size_t)3 * a.rows * a.lstride * sizeof(c2<T>);
    if (a.fixed && plan_is_576(a.plan))
      CHN_ROWS(a.rows, CHN_STAGED(T, m, hipLaunchKernelGGL((k_xpass<T, MV, 576, RZ>), grid, dim3(256), sh, st, a)));
    else if (a.fixed && plan_is_576c(a.plan))
      CHN_ROWS(a.rows, CHN_STAGED(T, m, hipLaunchKernelGGL((k_xpass<T, MV, kFn576Composite, RZ>), grid, dim3(256), sh, st, a)));
    else if (plan_is_composite(a.plan))
      CHN_ROWS(a.rows, CHN_STAGED(T, m, hipLaunchKernelGGL((k_xpass<T, MV, kFnComposite, RZ>), grid, dim3(256), sh, st, a)));
    else
      CHN_ROWS(a.rows, CHN_STAGED(T, m, hipLaunchKernelGGL((k_xpass<T, MV, 0, RZ>), grid, dim3(256), sh, st, a)));
    return hipGetLastError();
  }
  constexpr int QX = XrowCfg<T>::QX, XM = XrowCfg<T>::MV;
  const int nt = xrow_threads(a.d.p1, (int)sizeof(c2<T>));
  if (nt == 0 || !staging_fits(a.plan, 1, nt, XM)) return hipErrorInvalidValue;
  dim3 grid(a.d.p3, a.ny);
  const size_t sh = (size_t)a.d.p1 * sizeof(c2<T>);
  if (plan_is_composite(a.plan)) {
    if (nt == 256) hipLaunchKernelGGL((k_xrow<T, 256, QX, XM, kFnComposite>), grid, dim3(256), sh, st, a);
    else if (nt == 512) hipLaunchKernelGGL((k_xrow<T, 512, QX, XM, kFnComposite>), grid, dim3(512), sh, st, a);
    else hipLaunchKernelGGL((k_xrow<T, 1024, QX, XM, kFnComposite>), grid, dim3(1024), sh, st, a);
    return hipGetLastError();
  }
  if (nt == 256) hipLaunchKernelGGL((k_xrow<T, 256, QX, XM>), grid, dim3(256), sh, st, a);
  else if (nt == 512) hipLaunchKernelGGL((k_xrow<T, 512, QX, XM>), grid, dim3(512), sh, st, a);
  else if (nt == 1024 && a.fixed && plan_is_12288(a.plan))
    hipLaunchKernelGGL((k_xrow<T, 1024, QX, XM, 12288>), grid, dim3(1024), sh, st, a);
  else if (nt == 1024) hipLaunchKernelGGL((k_xrow<T, 1024, QX, XM>), grid, dim3(1024), sh, st, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

template hipError_t launch_xpass<float>(const XpassArgs<float>&, hipStream_t);

}  // namespace chn
