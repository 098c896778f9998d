// Version, status strings and the thread-local last-error message.
#include <string>

#include "common.hpp"

namespace csbfs {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int status, const std::string &msg) {
    g_last_error = msg;
    return status;
}

int hip_fail(hipError_t err, const char *what, const char *file, int line) {
    g_last_error = std::string(what) + " failed: " + hipGetErrorString(err) + " (" + file + ":" +
                   std::to_string(line) + ")";
    return CSBFS_EHIP;
}

}  // namespace csbfs

extern "C" int csbfs_version(void) { return CSBFS_VERSION; }

extern "C" const char *csbfs_strerror(int status) {
    switch (status) {
        case CSBFS_OK: return "ok";
        case CSBFS_EINVAL: return "invalid argument";
        case CSBFS_ERANGE: return "value out of range";
        case CSBFS_ENOSPACE: return "buffer or workspace too small";
        case CSBFS_EHIP: return "HIP runtime error";
        case CSBFS_EOVERFLOW: return "sub-block too large";
        case CSBFS_ECORRUPT: return "corrupt compressed stream";
        default: return "unknown status";
    }
}

extern "C" const char *csbfs_last_error(void) { return csbfs::g_last_error.c_str(); }
