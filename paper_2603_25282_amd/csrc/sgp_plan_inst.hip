// Instantiation of the pass and observables kernels of one (scalar type, register
// plan width) pair; the build compiles this file once per pair with
// -DSGP_INST_T=<float|double> -DSGP_INST_E=<4|8|12|16|24>.
#include "sgp_obs.hpp"

#if !defined(SGP_INST_T) || !defined(SGP_INST_E)
#error "compile with -DSGP_INST_T=<float|double> -DSGP_INST_E=<plan width>"
#endif

namespace sgp {
template hipError_t launch_pass_e<SGP_INST_T, SGP_INST_E>(int, void*, const PassArgs&, int, hipStream_t,
                                                           const hipEvent_t*);
template hipError_t launch_obs_e<SGP_INST_T, SGP_INST_E>(int, const void*, const PassArgs&, int, double*,
                                                         hipStream_t);
template hipError_t launch_batched_e<SGP_INST_T, SGP_INST_E>(int, const int2*, const PassArgs*, long, int,
                                                             hipStream_t);
}  // namespace sgp
