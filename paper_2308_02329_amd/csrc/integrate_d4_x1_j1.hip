// Instantiates the integrators for d = 4, 1 state term(s) and 1 coupling
// term(s): the register-resident kernels for every supported tile count and
// the streamed-J slab kernels for every tiles-per-wavefront bucket.
#include "integrate_slab.h"

namespace chym {
KernelSet lookup_resident_4_1_1(int tiles) { return lookup_tiles<4, 1, 1>(tiles); }
SlabKernels lookup_slab_4_1_1(int tpw, int waves, bool cp) { return slab_lookup_tpw<4, 1, 1>(tpw, waves, cp); }
}  // namespace chym
