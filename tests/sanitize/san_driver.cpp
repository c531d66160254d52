// Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the oracle's functions on
// small random sets (Pass-Join against brute force, every selection method, the banded against
// the full edit distance) and the library's check of caller-supplied host string sets on good
// and malformed inputs.  Exits 0 when every comparison holds; a sanitizer finding aborts.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "../../paper_1111_7171_amd/csrc/pj_validate.h"

extern "C" {
typedef struct {
    int64_t count;
    int32_t* a;
    int32_t* b;
    int64_t candidates, cells, selected, side_pairs;
    int64_t ncand;
    int32_t *cy, *cx, *ci, *cp, *cpass;
    int64_t* ccells;
    int64_t cap, ccap;
} orc_result;
int32_t orc_ed_full(const uint8_t* r, int32_t lr, const uint8_t* s, int32_t ls);
int32_t orc_ed_band(const uint8_t* r, int32_t lr, const uint8_t* s, int32_t ls, int32_t t);
orc_result* orc_self_join_pj(const uint8_t* chars, const int32_t* offs, int64_t n, int32_t tau,
                             int32_t tiebreak, int32_t probe_stride, int32_t probe_offset,
                             int32_t keep_cands, int32_t method);
orc_result* orc_join_pj(const uint8_t* rc, const int32_t* ro, int64_t rn, const uint8_t* sc,
                        const int32_t* so, int64_t sn, int32_t tau, int32_t keep_cands,
                        int32_t method, int32_t probe_stride, int32_t probe_offset);
orc_result* orc_self_join_bf(const uint8_t* chars, const int32_t* offs, int64_t n, int32_t tau,
                             int32_t nthreads);
orc_result* orc_join_bf(const uint8_t* rc, const int32_t* ro, int64_t rn, const uint8_t* sc,
                        const int32_t* so, int64_t sn, int32_t tau, int32_t nthreads);
void orc_result_free(orc_result* R);
}

static uint64_t g_state = 0x243F6A8885A308D3ull;
static uint64_t next_u64()     // SplitMix64
{
    uint64_t z = (g_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static int rnd(int n) { return (int)(next_u64() % (uint64_t)n); }

struct Set {
    std::vector<uint8_t> chars;
    std::vector<int32_t> offs{0};
    int64_t n() const { return (int64_t)offs.size() - 1; }
};

// random strings over `sigma` symbols with lengths 0..lmax, a share of them edited copies
static Set random_set(int n, int sigma, int lmax)
{
    Set S;
    std::vector<std::vector<uint8_t>> strs;
    for (int k = 0; k < n; ++k) {
        std::vector<uint8_t> s;
        if (!strs.empty() && rnd(3) == 0) {
            s = strs[(size_t)rnd((int)strs.size())];
            for (int e = rnd(4); e > 0; --e) {
                const int op = rnd(3), at = s.empty() ? 0 : rnd((int)s.size());
                if (op == 0 && !s.empty()) s[(size_t)at] = (uint8_t)('a' + rnd(sigma));
                else if (op == 1) s.insert(s.begin() + at, (uint8_t)('a' + rnd(sigma)));
                else if (!s.empty()) s.erase(s.begin() + at);
            }
        } else {
            for (int l = rnd(lmax + 1); l > 0; --l) s.push_back((uint8_t)('a' + rnd(sigma)));
        }
        strs.push_back(s);
        S.chars.insert(S.chars.end(), s.begin(), s.end());
        S.offs.push_back((int32_t)S.chars.size());
    }
    if (S.chars.empty()) S.chars.push_back(0);   // a valid pointer for empty sets
    return S;
}

static bool same_pairs(const orc_result* x, const orc_result* y)
{
    if (x->count != y->count) return false;
    for (int64_t k = 0; k < x->count; ++k)
        if (x->a[k] != y->a[k] || x->b[k] != y->b[k]) return false;
    return true;
}

static int failures = 0;
#define CHECK(c, ...)                                                    \
    do {                                                                 \
        if (!(c)) {                                                      \
            fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__);         \
            fprintf(stderr, __VA_ARGS__);                                \
            fprintf(stderr, "\n");                                       \
            ++failures;                                                  \
        }                                                                \
    } while (0)

int main()
{
    // banded distance (Sec. 5.1) against the full recurrence
    for (int trial = 0; trial < 4000; ++trial) {
        Set S = random_set(2, 2 + rnd(4), 24);
        const uint8_t* r = S.chars.data() + S.offs[0];
        const uint8_t* s = S.chars.data() + S.offs[1];
        const int lr = S.offs[1] - S.offs[0], ls = S.offs[2] - S.offs[1];
        const int full = orc_ed_full(r, lr, s, ls);
        for (int t = 0; t <= 6; ++t) {
            const int band = orc_ed_band(r, lr, s, ls, t);
            CHECK(band == (full <= t ? full : t + 1), "ed_band %d full %d t %d", band, full, t);
        }
    }
    // Pass-Join (Algorithm 1, every selection method) against brute force
    for (int trial = 0; trial < 24; ++trial) {
        const int sigma = 2 + trial % 5;
        Set S = random_set(120 + rnd(80), sigma, 18);
        Set R = random_set(60 + rnd(40), sigma, 18);
        for (int tau = 0; tau <= 4; ++tau) {
            orc_result* bf = orc_self_join_bf(S.chars.data(), S.offs.data(), S.n(), tau, 1);
            for (int method = 0; method < 4; ++method) {
                orc_result* pj = orc_self_join_pj(S.chars.data(), S.offs.data(), S.n(), tau,
                                                  trial & 1, 1, 0, method == 0, method);
                CHECK(same_pairs(pj, bf), "self-join trial %d tau %d method %d", trial, tau,
                      method);
                orc_result_free(pj);
            }
            orc_result_free(bf);
            orc_result* jb = orc_join_bf(R.chars.data(), R.offs.data(), R.n(), S.chars.data(),
                                         S.offs.data(), S.n(), tau, 1);
            orc_result* jp = orc_join_pj(R.chars.data(), R.offs.data(), R.n(), S.chars.data(),
                                         S.offs.data(), S.n(), tau, 1, 0, 1, 0);
            CHECK(same_pairs(jp, jb), "join trial %d tau %d", trial, tau);
            orc_result_free(jp);
            orc_result_free(jb);
        }
    }
    // the library's check of host string sets
    char msg[256];
    uint8_t bytes[8] = {'a', 'b', 'c', 'd', 'e', 'f', 'g', 'h'};
    int32_t good[4] = {0, 3, 3, 8};
    pj_strings s{3, bytes, good};
    CHECK(pj::check_host_strings(&s, "S", msg, sizeof msg) == PJ_OK, "good set: %s", msg);
    pj_strings empty{0, nullptr, good};
    CHECK(pj::check_host_strings(&empty, "S", msg, sizeof msg) == PJ_OK, "empty set: %s", msg);
    CHECK(pj::check_host_strings(nullptr, "S", msg, sizeof msg) == PJ_EINVAL, "null set");
    pj_strings neg{-1, bytes, good};
    CHECK(pj::check_host_strings(&neg, "S", msg, sizeof msg) == PJ_EINVAL, "n < 0");
    pj_strings nooffs{3, bytes, nullptr};
    CHECK(pj::check_host_strings(&nooffs, "S", msg, sizeof msg) == PJ_EINVAL, "null offsets");
    int32_t first[4] = {1, 3, 3, 8};
    pj_strings f{3, bytes, first};
    CHECK(pj::check_host_strings(&f, "S", msg, sizeof msg) == PJ_EINVAL, "offsets[0] != 0");
    int32_t dec[4] = {0, 5, 3, 8};
    pj_strings d{3, bytes, dec};
    CHECK(pj::check_host_strings(&d, "S", msg, sizeof msg) == PJ_EINVAL, "decreasing offsets");
    CHECK(strstr(msg, "offsets decrease at 1") != nullptr, "message: %s", msg);
    int32_t lng[3] = {0, 1, 1 + PJ_LEN_MAX + 1};
    pj_strings l{2, bytes, lng};
    CHECK(pj::check_host_strings(&l, "S", msg, sizeof msg) == PJ_ERANGE, "length > PJ_LEN_MAX");
    pj_strings nob{3, nullptr, good};
    CHECK(pj::check_host_strings(&nob, "S", msg, sizeof msg) == PJ_EINVAL, "null bytes");
    char tiny[4];
    CHECK(pj::check_host_strings(&d, "a long name", tiny, sizeof tiny) == PJ_EINVAL &&
              strlen(tiny) == 3, "truncated message");
    if (failures) {
        fprintf(stderr, "%d failures\n", failures);
        return 1;
    }
    printf("sanitized host checks passed\n");
    return 0;
}
