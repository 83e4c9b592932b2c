// Instantiates the integrators for d = 1, 3 state term(s) and 3 coupling
// term(s): the register-resident kernels for every supported tile count and
// the streamed-J slab kernels for every tiles-per-wavefront bucket.
#include "integrate_slab.h"

namespace chym {
KernelSet lookup_resident_1_3_3(int tiles) { return lookup_tiles<1, 3, 3>(tiles); }
SlabKernels lookup_slab_1_3_3(int tpw, int waves, bool cp) { return slab_lookup_tpw<1, 3, 3>(tpw, waves, cp); }
}  // namespace chym
