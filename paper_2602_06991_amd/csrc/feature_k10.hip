// The Top-K feature kernels instantiated for K = 10.
#include "feature_impl.hpp"

LGS_FEATURE_INSTANTIATE(10)
