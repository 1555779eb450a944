// Internal helpers shared by the library's translation units.
#pragma once
#include <cstdarg>
#include <cstdint>
#include <cstdio>

#include "../../include/mplayer.h"

// Record a thread-local error message (read back by mp_last_error) and
// return the code, so call sites read `return mp_fail(MP_EINVAL, "...")`.
int mp_fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
