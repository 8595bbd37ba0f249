// Library-wide entry points: version, error reporting, supported K.
#include "lgs_host.hpp"

namespace lgs {

static thread_local std::string g_error;

void set_error(const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_error = buf;
}

void clear_error() { g_error.clear(); }

}  // namespace lgs

extern "C" int lgs_abi_version(void) { return LGS_ABI_VERSION; }

extern "C" const char *lgs_last_error(void) { return lgs::g_error.c_str(); }

extern "C" const int32_t *lgs_supported_k(int32_t *count) {
    static const int32_t ks[] = {1, 2, 3, 4, 5, 8, 10, 16};
    if (count) *count = (int32_t)(sizeof(ks) / sizeof(ks[0]));
    return ks;
}
