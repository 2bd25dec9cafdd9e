// Error reporting of the library's host code (defined in capi.cpp, which
// also holds device calls) for the host-only sanitizer build of
// truncation.cpp: the message is kept, the status returned.
#include <string>

#include "arkcos_internal.h"

namespace arkcos {
static std::string g_msg;
void set_error(const std::string& msg) { g_msg = msg; }
arkcos_status_t fail(arkcos_status_t st, const std::string& msg) {
  g_msg = msg;
  return st;
}
}  // namespace arkcos
