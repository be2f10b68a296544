// Thread-local message of the last failed C-ABI call (cip_last_error), shared
// by the library's host translation units.
#pragma once
#include <string>

namespace cip {

inline thread_local std::string g_last_error;

inline int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

}  // namespace cip
