// The Top-K feature kernels instantiated for K = 2.
#include "feature_impl.hpp"

LGS_FEATURE_INSTANTIATE(2)
