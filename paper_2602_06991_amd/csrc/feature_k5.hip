// The Top-K feature kernels instantiated for K = 5.
#include "feature_impl.hpp"

LGS_FEATURE_INSTANTIATE(5)
