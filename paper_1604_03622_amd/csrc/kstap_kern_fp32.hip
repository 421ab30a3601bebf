// Instantiations of the narrow FP32 kernels (plain path).
#include "kstap_device.h"

namespace kstap {

#define KSTAP_ENTRY(P, Q, R, X) \
  {P, Q, R, X, X == 1, &launch_one<P, Q, R, X>, &launch_persist<P, Q, R, X>, \
   reinterpret_cast<const void*>(&kstap_persistent<P, Q, R, X>)}
// the table is a local static of a host function (a namespace-scope const
// array would also be emitted, unresolvable, for the device)
const Entry* entries_fp32(int* count) {
  static const Entry t[] = {
      KSTAP_ENTRY(2, 8, 4, 0),  KSTAP_ENTRY(2, 16, 4, 0), KSTAP_ENTRY(2, 32, 4, 0),
      KSTAP_ENTRY(3, 8, 4, 0),  KSTAP_ENTRY(3, 8, 8, 0),  KSTAP_ENTRY(3, 12, 4, 0), KSTAP_ENTRY(3, 12, 8, 0),
      KSTAP_ENTRY(3, 16, 4, 0), KSTAP_ENTRY(3, 16, 8, 0), KSTAP_ENTRY(4, 8, 4, 0),  KSTAP_ENTRY(4, 16, 4, 0),
      KSTAP_ENTRY(6, 8, 4, 0),
  };
  *count = int(sizeof(t) / sizeof(t[0]));
  return t;
}
#undef KSTAP_ENTRY

}  // namespace kstap
