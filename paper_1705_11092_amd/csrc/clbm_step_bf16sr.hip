// clbm_step_bf16sr.hip -- step and batch kernels for BF16 with stochastic rounding storage.
#include "clbm_step.h"
#include "clbm_step2.h"

namespace clbm {
template hipError_t launch_step_st<ST_BF16_SR>(const LatDesc &, int, int, size_t, hipStream_t);
template hipError_t launch_resident_st<ST_BF16_SR>(const LatDesc &, int, int, hipStream_t);
template hipError_t launch_step2_st<ST_BF16_SR>(const LatDesc &, int, hipStream_t);
template hipError_t launch_batch2_st<ST_BF16_SR>(const LatDesc *, const int32_t *, int64_t, int, bool, int,
                                          int, int, hipStream_t);
template hipError_t launch_batch_st<ST_BF16_SR>(const LatDesc *, const int32_t *, int64_t, int, int,
                                         int, int, size_t, hipStream_t);
}  // namespace clbm
