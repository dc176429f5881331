// pdn_elem_full.hip -- the element / node kernel with full 2x2x2 Gauss
// integration of the bulk elements (Section 2): eight damage states per
// element, no hourglass control.
#include "pdn_elem.h"

namespace pdn {

template <typename R>
hipError_t launch_elem_node_full(const ElemArgs<R> &a, int tile, hipStream_t s)
{
    return launch_elem_node_full_v<R>(a, tile, s);
}
template hipError_t launch_elem_node_full<float>(const ElemArgs<float> &, int, hipStream_t);
template hipError_t launch_elem_node_full<double>(const ElemArgs<double> &, int, hipStream_t);

template <typename R>
hipError_t launch_elem_node_batch_full(const ElemArgs<R> *args, const int *start, int ncase, int nblocks, int tile,
                                       hipStream_t s)
{
    return launch_elem_node_batch_full_v<R>(args, start, ncase, nblocks, tile, s);
}
template hipError_t launch_elem_node_batch_full<float>(const ElemArgs<float> *, const int *, int, int, int,
                                                       hipStream_t);
template hipError_t launch_elem_node_batch_full<double>(const ElemArgs<double> *, const int *, int, int, int,
                                                        hipStream_t);

}  // namespace pdn
