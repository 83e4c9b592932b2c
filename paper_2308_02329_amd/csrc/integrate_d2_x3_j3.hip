// Instantiates the register-resident integrator for d = 2, 3 state
// term(s) and 3 coupling term(s), every supported tile count.
#include "integrate_kernel.h"

namespace chym {
KernelSet lookup_resident_2_3_3(int tiles) { return lookup_tiles<2, 3, 3>(tiles); }
}  // namespace chym
