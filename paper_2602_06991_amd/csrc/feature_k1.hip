// The Top-K feature kernels instantiated for K = 1.
#include "feature_impl.hpp"

LGS_FEATURE_INSTANTIATE(1)
