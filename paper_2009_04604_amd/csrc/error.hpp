// Thread-local error message shared by every C-ABI entry point.
#pragma once
#include <string>

namespace lbm {
// Record `msg` as the calling thread's last error and return `code`.
int set_error(int code, const std::string& msg);
void clear_error();
}  // namespace lbm
