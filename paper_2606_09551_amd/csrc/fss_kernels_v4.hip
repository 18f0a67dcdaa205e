// Instantiates the kernels for AES variant 4 (the fixed-key PRG bitsliced in
// registers; the dealer's keyed randomness on table layout 1).
#include "fss_kernels_impl.hpp"

namespace fss {
template struct VariantOps<4>;
}
