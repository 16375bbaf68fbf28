// Thread-local error message shared by the library's translation units.
#pragma once
#include <cstdarg>
#include <cstdio>

extern "C" const char *rbicg_last_error(void);

// Record a formatted message as the calling thread's last error; returns code.
int rbicg_fail(int code, const char *fmt, ...);
