// The Top-K feature kernels instantiated for K = 3.
#include "feature_impl.hpp"

LGS_FEATURE_INSTANTIATE(3)
