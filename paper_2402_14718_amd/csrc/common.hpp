// Shared host-side helpers of the sbtrack library: status reporting and
// host-side argument checks.
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

// Full check of a host QUBO (validate.cpp): n >= 1; row_ptr non-decreasing
// within [0, nnz] (checked for every row before any row is read); columns
// in range, ascending, off the diagonal; finite a and b; b symmetric.
// `what` names the QUBO in messages ("qubo", "event 3").  *max_row (may be
// NULL) receives the longest row.  SBT_OK or SBT_EINVAL.
int validate_qubo_host(const sbt_qubo *q, const char *who, const char *what, int32_t *max_row);

// The array structure alone (n >= 0 allowed; row_ptr non-decreasing from 0
// to nnz, columns in range): what reading every row safely needs.
int validate_qubo_structure(const sbt_qubo *q, const char *who, const char *what);

}  // namespace sbt
