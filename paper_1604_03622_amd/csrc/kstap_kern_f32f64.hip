// Instantiations of the narrow kernels with FP32 covariance and FP64 solves
// (full covariance sums, no sliding window): the precision for frames with
// strong point scatterers, where FP32 eigensolves lose the clutter subspace.
#include "kstap_device.h"

namespace kstap {

#define KSTAP_ENTRY(P, Q, R, X) \
  {P, Q, R, X, false, &launch_one<P, Q, R, X>, &launch_persist<P, Q, R, X>, \
   reinterpret_cast<const void*>(&kstap_persistent<P, Q, R, X>)}
// the table is a local static of a host function (a namespace-scope const
// array would also be emitted, unresolvable, for the device)
const Entry* entries_f32f64(int* count) {
  static const Entry t[] = {
      KSTAP_ENTRY(3, 8, 4, 2),
      KSTAP_ENTRY(3, 16, 4, 2),
  };
  *count = int(sizeof(t) / sizeof(t[0]));
  return t;
}
#undef KSTAP_ENTRY

}  // namespace kstap
