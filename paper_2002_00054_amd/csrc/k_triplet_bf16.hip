// Instantiation of the pair/triplet kernels for one arithmetic form.
#include "kernels.h"
#include "k_triplet.inc"

namespace nnp {
template void launch_triplet<P_BF16>(int, int, const TripArgs<P_BF16>&, hipStream_t);
template size_t triplet_lds_bytes<P_BF16>(int, int, int, int);
}  // namespace nnp
