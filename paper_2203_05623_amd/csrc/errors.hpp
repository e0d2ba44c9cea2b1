// Error reporting of the C-ABI: status codes plus a thread-local message.
#pragma once

#include "../../include/sth.h"

namespace sth {

// Formats the thread-local message returned by sth_last_error().
void set_error(const char* fmt, ...) __attribute__((format(printf, 1, 2)));

// Carries a status code from deep inside the library to the C-ABI boundary,
// where it is converted to the return value (no exception crosses the ABI).
struct Error {
  int code;
  explicit Error(int c) : code(c) {}
};

}  // namespace sth
