// Shared host-side helpers of the sbtrack library: status reporting.
#pragma once

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "sbtrack.h"

namespace sbt {

// Records a formatted message for sbt_last_error() and returns `code`.
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

// Clears the thread-local message.
void clear_error();


// Argument checks shared by the host and GPU QUBO builders: fills *p (the
// defaults when pp is NULL), clears *out; SBT_OK or an error status.
int check_build_inputs(const sbt_hit *hits, int64_t n_hits, const sbt_build_params *pp,
                       sbt_qubo **out, sbt_build_params *p, const char *who);

}  // namespace sbt
