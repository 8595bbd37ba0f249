// The Top-K feature kernels instantiated for K = 16.
#include "feature_impl.hpp"

LGS_FEATURE_INSTANTIATE(16)
