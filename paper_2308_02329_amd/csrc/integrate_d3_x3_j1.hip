// Instantiates the integrators for d = 3, 3 state term(s) and 1 coupling
// term(s): the register-resident kernels for every supported tile count and
// the streamed-J slab kernels for every tiles-per-wavefront bucket.
#include "integrate_slab.h"

namespace chym {
KernelSet lookup_resident_3_3_1(int tiles) { return lookup_tiles<3, 3, 1>(tiles); }
SlabKernels lookup_slab_3_3_1(int tpw, int waves, bool cp) { return slab_lookup_tpw<3, 3, 1>(tpw, waves, cp); }
}  // namespace chym
