// Instantiates the register-resident integrator for d = 1, 3 state
// term(s) and 3 coupling term(s), every supported tile count.
#include "integrate_kernel.h"

namespace chym {
KernelSet lookup_resident_1_3_3(int tiles) { return lookup_tiles<1, 3, 3>(tiles); }
}  // namespace chym
