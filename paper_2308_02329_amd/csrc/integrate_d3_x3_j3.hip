// Instantiates the register-resident integrator for d = 3, 3 state
// term(s) and 3 coupling term(s), every supported tile count.
#include "integrate_kernel.h"

namespace chym {
KernelSet lookup_resident_3_3_3(int tiles) { return lookup_tiles<3, 3, 3>(tiles); }
}  // namespace chym
