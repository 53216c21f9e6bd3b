// Launch dispatch of the split-step kernels (the kernels themselves are in
// sgp_passes.hpp and, for the observables, sgp_obs.hpp): line length and register plan -> the instantiation compiled in
// sgp_plan_inst.hip for that plan width; the batched ensemble passes; the
// propagator tables.
#include "sgp_obs.hpp"

namespace sgp {

#define SGP_EXTERN(TT, EE)                                                                            \
  extern template hipError_t launch_pass_e<TT, EE>(int, void*, const PassArgs&, int, hipStream_t, const hipEvent_t*);   \
  extern template hipError_t launch_obs_e<TT, EE>(int, const void*, const PassArgs&, int, double*, hipStream_t);
SGP_EXTERN(float, 4) SGP_EXTERN(float, 8) SGP_EXTERN(float, 12) SGP_EXTERN(float, 16) SGP_EXTERN(float, 24)
SGP_EXTERN(double, 4) SGP_EXTERN(double, 8) SGP_EXTERN(double, 12) SGP_EXTERN(double, 16) SGP_EXTERN(double, 24)
#undef SGP_EXTERN
#define SGP_EXTERN_B(TT, EE) \
  extern template hipError_t launch_batched_e<TT, EE>(int, const int2*, const PassArgs*, long, int, hipStream_t);
SGP_EXTERN_B(float, 4) SGP_EXTERN_B(float, 8) SGP_EXTERN_B(float, 12) SGP_EXTERN_B(float, 16) SGP_EXTERN_B(float, 24)
SGP_EXTERN_B(double, 4) SGP_EXTERN_B(double, 8) SGP_EXTERN_B(double, 12) SGP_EXTERN_B(double, 16)
#undef SGP_EXTERN_B

template <typename T>
hipError_t launch_pass(int kind, void* psi, const PassArgs& a, int n, int e, hipStream_t st, const hipEvent_t* ev) {
  if (!plan_ok(n, e, (int)sizeof(T))) return hipErrorInvalidValue;
  switch (e) {
    case 4: return launch_pass_e<T, 4>(kind, psi, a, n, st, ev);
    case 8: return launch_pass_e<T, 8>(kind, psi, a, n, st, ev);
    case 12: return launch_pass_e<T, 12>(kind, psi, a, n, st, ev);
    case 16: return launch_pass_e<T, 16>(kind, psi, a, n, st, ev);
    case 24: return launch_pass_e<T, 24>(kind, psi, a, n, st, ev);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_obs(int kind, const void* psi, const PassArgs& a, int n, int e, double* part, hipStream_t st) {
  if (!plan_ok(n, e, (int)sizeof(T))) return hipErrorInvalidValue;
  switch (e) {
    case 4: return launch_obs_e<T, 4>(kind, psi, a, n, part, st);
    case 8: return launch_obs_e<T, 8>(kind, psi, a, n, part, st);
    case 12: return launch_obs_e<T, 12>(kind, psi, a, n, part, st);
    case 16: return launch_obs_e<T, 16>(kind, psi, a, n, part, st);
    case 24: return launch_obs_e<T, 24>(kind, psi, a, n, part, st);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// Deterministic sum of block partials: block q adds part[b nq + q] over b; thread t
// takes b = t, t + 256, ... in order, then a fixed pairwise tree over the threads.
// The order does not depend on timing, so repeated calls give bitwise equal sums.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ part, long nb, int nq,
                                                      double* __restrict__ out) {
  __shared__ double red[256];
  const int q = blockIdx.x, t = threadIdx.x;
  double s = 0.0;
  for (long b = t; b < nb; b += 256) s += part[b * nq + q];
  red[t] = s;
  __syncthreads();
#pragma unroll
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  if (t == 0) out[q] = red[0];
}

hipError_t launch_sum_partials(const double* part, long nb, int nq, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_partials, dim3((unsigned)nq), dim3(256), 0, st, part, nb, nq, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_build_tables(void* cs, void* kin_x, void* kin_y, void* kin_z, const int* n, const double* L,
                               int dim, double Omega, double gamma, double d, hipStream_t st) {
  const long nxy = (long)n[0] * n[1];
  hipLaunchKernelGGL((k_build_cs<T>), dim3((unsigned)((nxy + 255) / 256)), dim3(256), 0, st, (T*)cs, n[0], n[1],
                     L[0], L[1], Omega, gamma, d);
  hipLaunchKernelGGL((k_build_kin<T>), dim3((n[0] + 255) / 256), dim3(256), 0, st, (cx<T>*)kin_x, n[0], L[0], d);
  hipLaunchKernelGGL((k_build_kin<T>), dim3((n[1] + 255) / 256), dim3(256), 0, st, (cx<T>*)kin_y, n[1], L[1], d);
  if (dim == 3)
    hipLaunchKernelGGL((k_build_kin<T>), dim3((n[2] + 255) / 256), dim3(256), 0, st, (cx<T>*)kin_z, n[2], L[2], d);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_pass_batched(int kind, int e, const void* items, const void* args, long nitems, int nmax,
                               hipStream_t st) {
  const int2* it = (const int2*)items;
  const PassArgs* ar = (const PassArgs*)args;
  if (nitems <= 0) return hipSuccess;
  switch (e) {
    case 4: return launch_batched_e<T, 4>(kind, it, ar, nitems, nmax, st);
    case 8: return launch_batched_e<T, 8>(kind, it, ar, nitems, nmax, st);
    case 12: return launch_batched_e<T, 12>(kind, it, ar, nitems, nmax, st);
    case 16: return launch_batched_e<T, 16>(kind, it, ar, nitems, nmax, st);
    case 24:
      if constexpr (sizeof(T) == 4) return launch_batched_e<T, 24>(kind, it, ar, nitems, nmax, st);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_pass_batched<float>(int, int, const void*, const void*, long, int, hipStream_t);
template hipError_t launch_pass_batched<double>(int, int, const void*, const void*, long, int, hipStream_t);
template hipError_t launch_pass<float>(int, void*, const PassArgs&, int, int, hipStream_t, const hipEvent_t*);
template hipError_t launch_pass<double>(int, void*, const PassArgs&, int, int, hipStream_t, const hipEvent_t*);
template hipError_t launch_obs<float>(int, const void*, const PassArgs&, int, int, double*, hipStream_t);
template hipError_t launch_obs<double>(int, const void*, const PassArgs&, int, int, double*, hipStream_t);
template hipError_t launch_build_tables<float>(void*, void*, void*, void*, const int*, const double*, int, double,
                                               double, double, hipStream_t);
template hipError_t launch_build_tables<double>(void*, void*, void*, void*, const int*, const double*, int, double,
                                                double, double, hipStream_t);

}  // namespace sgp
