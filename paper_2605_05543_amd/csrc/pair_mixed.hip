// pair_mixed.hip -- mixed-precision pair kernel (not built yet).
#include "empp_dev.h"

namespace empp {

extern const bool kHaveMixed = false;

hipError_t launch_pair_mixed(const PairParams &, hipStream_t, bool, bool) { return hipErrorInvalidValue; }

}  // namespace empp
