// pj_validate.h -- checks of caller-supplied host string sets, with no HIP dependency (so that
// they also build into a sanitizer run of plain host code).
#pragma once

#include <stddef.h>

#include "../../include/passjoin.h"

namespace pj {

// PJ_OK when S is a valid host string set (the pj_strings contract: n >= 0 and below 2^31 - 1,
// offsets[0] == 0, non-decreasing offsets, lengths <= PJ_LEN_MAX, bytes non-NULL when
// offsets[n] > 0); otherwise the error code, with a message naming `what` written to msg (at
// most cap bytes, NUL-terminated).  Reads offsets[0 .. n] and nothing else.
int check_host_strings(const pj_strings* S, const char* what, char* msg, size_t cap);

}  // namespace pj
