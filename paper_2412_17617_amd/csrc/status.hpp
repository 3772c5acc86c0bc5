// Error reporting shared by the C ABI entry points.
#pragma once

#include <string>

namespace pxd {

// Records msg as the calling thread's last error and returns rc.
int set_thread_error(int rc, const std::string& msg);
const char* thread_error();

}  // namespace pxd
