// pdn_elem_sur.hip -- the element / node kernel with the constitutive
// surrogate network (plies of law 2 evaluate it on the matrix cores).
#include "pdn_elem.h"

namespace pdn {

template <typename R>
hipError_t launch_elem_node_sur(const ElemArgs<R> &a, int tile, hipStream_t s)
{
    return launch_elem_node_v<R, true>(a, tile, s);
}
template hipError_t launch_elem_node_sur<float>(const ElemArgs<float> &, int, hipStream_t);
template hipError_t launch_elem_node_sur<double>(const ElemArgs<double> &, int, hipStream_t);

template <typename R>
hipError_t launch_elem_node_sur_wide(const ElemArgs<R> &a, int tile, hipStream_t s)
{
    return launch_elem_node_sur_wide_v<R>(a, tile, s);
}
template hipError_t launch_elem_node_sur_wide<float>(const ElemArgs<float> &, int, hipStream_t);
template hipError_t launch_elem_node_sur_wide<double>(const ElemArgs<double> &, int, hipStream_t);

template <typename R>
hipError_t launch_elem_node_batch_sur(const ElemArgs<R> *args, const int *start, int ncase, int nblocks, int tile,
                                      hipStream_t s)
{
    return launch_elem_node_batch_v<R, true>(args, start, ncase, nblocks, tile, s);
}
template hipError_t launch_elem_node_batch_sur<float>(const ElemArgs<float> *, const int *, int, int, int,
                                                      hipStream_t);
template hipError_t launch_elem_node_batch_sur<double>(const ElemArgs<double> *, const int *, int, int, int,
                                                       hipStream_t);

int elem_node_lds_bytes_sur(int mixed, int tile) { return mixed ? lds_v<float, true>(tile) : lds_v<double, true>(tile); }

}  // namespace pdn
