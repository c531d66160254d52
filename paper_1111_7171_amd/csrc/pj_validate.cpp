// pj_validate.cpp -- checks of caller-supplied host string sets (no HIP dependency).
#include "pj_validate.h"

#include <stdint.h>
#include <stdio.h>

namespace pj {

int check_host_strings(const pj_strings* S, const char* what, char* msg, size_t cap)
{
    if (cap > 0) msg[0] = '\0';
    if (!S) {
        snprintf(msg, cap, "%s: null pj_strings", what);
        return PJ_EINVAL;
    }
    if (S->n < 0) {
        snprintf(msg, cap, "%s: n < 0", what);
        return PJ_EINVAL;
    }
    if (S->n >= (int64_t)INT32_MAX) {
        snprintf(msg, cap, "%s: too many strings", what);
        return PJ_ERANGE;
    }
    if (!S->offsets) {
        snprintf(msg, cap, "%s: null offsets", what);
        return PJ_EINVAL;
    }
    if (S->offsets[0] != 0) {
        snprintf(msg, cap, "%s: offsets[0] != 0", what);
        return PJ_EINVAL;
    }
    for (int64_t k = 0; k < S->n; ++k) {
        const int64_t l = (int64_t)S->offsets[k + 1] - S->offsets[k];
        if (l < 0) {
            snprintf(msg, cap, "%s: offsets decrease at %lld", what, (long long)k);
            return PJ_EINVAL;
        }
        if (l > PJ_LEN_MAX) {
            snprintf(msg, cap, "%s: string %lld has length %lld > %d", what, (long long)k,
                     (long long)l, PJ_LEN_MAX);
            return PJ_ERANGE;
        }
    }
    if (S->offsets[S->n] > 0 && !S->bytes) {
        snprintf(msg, cap, "%s: null bytes", what);
        return PJ_EINVAL;
    }
    return PJ_OK;
}

}  // namespace pj
