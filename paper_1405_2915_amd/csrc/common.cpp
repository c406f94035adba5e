#include "common.hpp"

#include <cstdarg>
#include <cstdio>

namespace skel {

namespace {
thread_local char t_msg[512] = "";
Runtime g_runtime;
}  // namespace

Runtime& rt() { return g_runtime; }

skel_status fail(skel_status st, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(t_msg, sizeof t_msg, fmt, ap);
    va_end(ap);
    return st;
}

void clear_error() { t_msg[0] = '\0'; }

const char* dtype_name(skel_dtype t) {
    switch (t) {
    case SKEL_F32: return "f32";
    case SKEL_BF16: return "bf16";
    case SKEL_I32: return "i32";
    case SKEL_I64: return "i64";
    }
    return "?";
}

}  // namespace skel

extern "C" const char* skel_last_error(void) { return skel::t_msg; }
