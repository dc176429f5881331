// pdn_elem_plas.hip -- the element / node kernel with the matrix shear
// plasticity of the intralaminar law (Section 2.3.1, Algorithm 4's first two
// lines): one-point elements whose plies carry a plastic state.  Its own
// translation unit, so that the plain kernel keeps its register budget.
#include "pdn_elem.h"

namespace pdn {

template <typename R>
hipError_t launch_elem_node_plas(const ElemArgs<R> &a, int tile, hipStream_t s)
{
    return launch_elem_node_plas_v<R>(a, tile, s);
}
template hipError_t launch_elem_node_plas<float>(const ElemArgs<float> &, int, hipStream_t);
template hipError_t launch_elem_node_plas<double>(const ElemArgs<double> &, int, hipStream_t);

}  // namespace pdn
