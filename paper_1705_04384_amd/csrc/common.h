// Internal helpers shared by the library's translation units (host side).
#pragma once

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "fdgmres.h"

namespace fdg {

// Records a message for fdg_last_error() in the calling thread and returns the status.
int set_error(int status, const char *fmt, ...);
void clear_error();

inline int64_t ipow(int64_t b, int e) {
  int64_t r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

}  // namespace fdg
