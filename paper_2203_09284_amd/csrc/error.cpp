// Thread-local error message of the C ABI.
#include <stdarg.h>
#include <stdio.h>

#include <string>

#include "internal.h"

static thread_local std::string g_last_error;

int pr_fail(int code, const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

void pr_clear_error() { g_last_error.clear(); }

extern "C" const char *pr_last_error(void) { return g_last_error.c_str(); }
