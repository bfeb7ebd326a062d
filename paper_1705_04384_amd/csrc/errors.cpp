// Status strings and the per-thread last-error message of the C ABI.
#include <cstdarg>
#include <cstdio>

#include "common.h"

namespace fdg {

static thread_local char g_last_error[512] = "";

int set_error(int status, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
  return status;
}

void clear_error() { g_last_error[0] = '\0'; }

}  // namespace fdg

extern "C" const char *fdg_last_error(void) { return fdg::g_last_error; }

extern "C" const char *fdg_status_str(int status) {
  switch (status) {
    case FDG_OK: return "FDG_OK";
    case FDG_NOT_CONVERGED: return "FDG_NOT_CONVERGED";
    case FDG_EINVAL: return "FDG_EINVAL";
    case FDG_ENOMEM: return "FDG_ENOMEM";
    case FDG_EHIP: return "FDG_EHIP";
    case FDG_ECOMPLEX: return "FDG_ECOMPLEX";
    case FDG_ENOTREADY: return "FDG_ENOTREADY";
    case FDG_ENOCONV: return "FDG_ENOCONV";
    case FDG_EFULL: return "FDG_EFULL";
    default: return "FDG_UNKNOWN";
  }
}
