// pdn_elem_full_plas.hip -- the element / node kernel with full 2x2x2 Gauss
// integration and the matrix shear plasticity of the intralaminar law
// (Section 2; Section 2.3.1, Algorithm 4's first two lines): eight damage
// states and eight plastic states per element.  Its own translation unit, so
// that the build of the other variants is unchanged.
#include "pdn_elem.h"

namespace pdn {

template <typename R>
hipError_t launch_elem_node_full_plas(const ElemArgs<R> &a, int tile, hipStream_t s)
{
    return launch_elem_node_full_v<R, true>(a, tile, s);
}
template hipError_t launch_elem_node_full_plas<float>(const ElemArgs<float> &, int, hipStream_t);
template hipError_t launch_elem_node_full_plas<double>(const ElemArgs<double> &, int, hipStream_t);

}  // namespace pdn
