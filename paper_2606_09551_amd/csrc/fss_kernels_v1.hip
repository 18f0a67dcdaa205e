// Instantiates the kernels for AES table layout 1.
#include "fss_kernels_impl.hpp"

namespace fss {
template struct VariantOps<1>;
}
