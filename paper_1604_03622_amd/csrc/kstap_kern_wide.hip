// Instantiations of the wide-pixel kernels (p*q > 64), both precisions.
#include "kstap_device.h"

namespace kstap {

#define KSTAP_ENTRY(P, Q, R, X) \
  {P, Q, R, X, X == 1, &launch_one<P, Q, R, X>, &launch_persist<P, Q, R, X>, \
   reinterpret_cast<const void*>(&kstap_persistent<P, Q, R, X>)}
// wide pixels: one 4-wave workgroup per pixel (no persistent form)
// the table is a local static of a host function (a namespace-scope const
// array would also be emitted, unresolvable, for the device)
const Entry* entries_wide(int* count) {
  static const Entry t[] = {
      {5, 24, 4, 0, false, &launch_wide<5, 24, 4, 0>, nullptr, nullptr},
      {5, 24, 4, 1, false, &launch_wide<5, 24, 4, 1>, nullptr, nullptr},
      {6, 16, 4, 0, false, &launch_wide<6, 16, 4, 0>, nullptr, nullptr},
      {6, 16, 4, 1, false, &launch_wide<6, 16, 4, 1>, nullptr, nullptr},
  };
  *count = int(sizeof(t) / sizeof(t[0]));
  return t;
}
#undef KSTAP_ENTRY

}  // namespace kstap
