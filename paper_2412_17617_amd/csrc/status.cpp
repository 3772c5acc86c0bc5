// Thread-local last-error string for calls made without a context.
#include "status.hpp"

namespace pxd {
namespace {
thread_local std::string g_error;
}

int set_thread_error(int rc, const std::string& msg) {
  g_error = msg;
  return rc;
}

const char* thread_error() { return g_error.c_str(); }

}  // namespace pxd
