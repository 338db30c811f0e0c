// Joint BF apply instantiations for float, 5 columns (the last one from the second source).
#include "apply_bf_impl.h"

namespace gsf {
template <typename T, int M>
void bf_apply_joint_tm(const bfk::ApplyArgs& a, int ndim, int r, int rpt, hipStream_t s, int* nb) {
  bfk::launch_bf_r<T, M, 1>(a, ndim, r, rpt, s, nb);
}
template void bf_apply_joint_tm<float, 5>(const bfk::ApplyArgs&, int, int, int, hipStream_t, int*);
}  // namespace gsf
