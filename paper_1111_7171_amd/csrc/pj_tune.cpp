// Autotuner for the batched path's launch parameters (persistent verification grid, list
// segments per wave chunk, the small/large inverted-list threshold, probe grid and thread
// mapping).  None of them
// changes a result: they decide only how the candidates of Algorithm 1 are spread over waves.
//
// Parameters are kept per (GPU architecture, tau, length bucket), the bucket being the bit
// length of the probe set's rounded mean string length.  pj_tune searches them by coordinate
// descent on a caller-supplied workload, timing the probe and verification phases with hip
// events; the result goes to an in-process table and, when pj_options.tune_cache names a file,
// to that file, which later calls read back.  The file is plain text:
//
//   # passjoin tune cache v3: arch tau len_bucket verify_waves_per_cu seg_chunk big_list
//   #   probe_blocks_per_cu lane_cands probe_map ms
//   gfx950 4 4 32 4 32 8 2 0 112.300
//
// Lines of the v2 format (without probe_map) read as probe_map 0.  Unknown or out-of-range
// lines are ignored.  A file that changes on disk is read again.
#include <sys/stat.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "pj_host_internal.h"

namespace pj {

namespace {

using Key = std::tuple<std::string, int, int>;   // arch, tau, length bucket

struct Entry {
    TuneParams p;
    double ms = 0.0;
};

struct FileState {
    long long mtime_ns = -1;
    long long size = -1;
    std::map<Key, Entry> table;
};

std::mutex g_mu;
std::map<Key, Entry> g_local;                  // tuned in this process without a cache file
std::map<std::string, FileState> g_files;      // cache file path -> parsed contents

const int kWavesOpts[] = {8, 16, 32, 64, 128, 256, 512, 1024};
const int kChunkOpts[] = {1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048};
const int kBigOpts[] = {16, 32, 64, 128};
const int kProbeOpts[] = {4, 8, 16};
const int kLaneOpts[] = {1, 2};
const int kMapOpts[] = {0, 1};

template <size_t N>
bool in(const int (&opts)[N], int v)
{
    return std::find(std::begin(opts), std::end(opts), v) != std::end(opts);
}

std::string arch_name()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        (void)hipGetLastError();
        return "unknown";
    }
    std::string a = prop.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

int length_bucket(double mean_len)
{
    long long m = (long long)(mean_len + 0.5);
    int b = 0;
    while (m > 0) {
        ++b;
        m >>= 1;
    }
    return b;
}

bool stat_file(const char* path, long long& mtime_ns, long long& size)
{
    struct stat sb;
    if (stat(path, &sb) != 0) return false;
    mtime_ns = (long long)sb.st_mtim.tv_sec * 1000000000LL + sb.st_mtim.tv_nsec;
    size = (long long)sb.st_size;
    return true;
}

void parse_file(const char* path, std::map<Key, Entry>& table)
{
    table.clear();
    FILE* f = fopen(path, "r");
    if (!f) return;
    char line[512];
    while (fgets(line, sizeof line, f)) {
        if (line[0] == '#') continue;
        char arch[128];
        int tau, lb;
        Entry e;
        const int got = sscanf(line, "%127s %d %d %d %d %d %d %d %d %lf", arch, &tau, &lb,
                               &e.p.verify_waves_per_cu, &e.p.seg_chunk, &e.p.big_list,
                               &e.p.probe_blocks_per_cu, &e.p.lane_cands, &e.p.probe_map, &e.ms);
        if (got != 10) {
            // v2: no probe_map column
            e.p.probe_map = 0;
            if (sscanf(line, "%127s %d %d %d %d %d %d %d %lf", arch, &tau, &lb,
                       &e.p.verify_waves_per_cu, &e.p.seg_chunk, &e.p.big_list,
                       &e.p.probe_blocks_per_cu, &e.p.lane_cands, &e.ms) != 9)
                continue;
        }
        if (tau < 0 || tau > kTauMax || lb < 0 || lb > 12 || !tune_params_valid(e.p)) continue;
        table[Key(arch, tau, lb)] = e;
    }
    fclose(f);
}

// the table of a cache file, read again when the file changed
std::map<Key, Entry>& file_table(const char* path)
{
    FileState& fs = g_files[path];
    long long mt = -1, sz = -1;
    if (!stat_file(path, mt, sz)) {
        fs.table.clear();
        fs.mtime_ns = fs.size = -1;
    } else if (mt != fs.mtime_ns || sz != fs.size) {
        parse_file(path, fs.table);
        fs.mtime_ns = mt;
        fs.size = sz;
    }
    return fs.table;
}

void write_file(const char* path, const std::map<Key, Entry>& table)
{
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "w");
    if (!f) throw Error(PJ_EINVAL, "cannot write tune cache %s", path);
    fprintf(f, "# passjoin tune cache v3: arch tau len_bucket verify_waves_per_cu seg_chunk "
               "big_list probe_blocks_per_cu lane_cands probe_map ms\n");
    for (const auto& kv : table) {
        const Entry& e = kv.second;
        fprintf(f, "%s %d %d %d %d %d %d %d %d %.3f\n", std::get<0>(kv.first).c_str(),
                std::get<1>(kv.first), std::get<2>(kv.first), e.p.verify_waves_per_cu,
                e.p.seg_chunk, e.p.big_list, e.p.probe_blocks_per_cu, e.p.lane_cands,
                e.p.probe_map, e.ms);
    }
    if (fclose(f) != 0 || rename(tmp.c_str(), path) != 0)
        throw Error(PJ_EINVAL, "cannot write tune cache %s", path);
}

double mean_length(const pj_strings* S)
{
    return S->n > 0 ? (double)(S->offsets[S->n] - S->offsets[0]) / (double)S->n : 0.0;
}

}  // namespace

bool tune_params_valid(const TuneParams& p)
{
    return in(kWavesOpts, p.verify_waves_per_cu) && in(kChunkOpts, p.seg_chunk) &&
           in(kBigOpts, p.big_list) && in(kProbeOpts, p.probe_blocks_per_cu) &&
           in(kLaneOpts, p.lane_cands) && in(kMapOpts, p.probe_map);
}

TuneParams tune_lookup(const char* cache, int tau, double mean_len)
{
    const Key k(arch_name(), tau, length_bucket(mean_len));
    std::lock_guard<std::mutex> lk(g_mu);
    if (cache && cache[0]) {
        const auto& t = file_table(cache);
        const auto it = t.find(k);
        if (it != t.end()) return it->second.p;
    }
    const auto it = g_local.find(k);
    return it != g_local.end() ? it->second.p : TuneParams{};
}

// Device time (ms) of the probe and verification phases of one self-join under p; the pairs
// are checked against the first run's count, since no parameter may change the result.
static double time_one(const pj_strings* S, int32_t tau, const pj_options* base,
                       const TuneParams& p, int64_t* pairs);

}  // namespace pj

using namespace pj;

extern "C" {

int pj_tune(const pj_strings* S, int32_t tau, const pj_options* opt, pj_tune_result* out)
{
    try {
        if (!out) throw Error(PJ_EINVAL, "null result");
        memset(out, 0, sizeof *out);
        if (tau < 0 || tau > kTauMax) throw Error(PJ_EINVAL, "tau %d outside [0, %d]", tau, kTauMax);
        if (opt && opt->inputs_on_device) throw Error(PJ_EINVAL, "pj_tune takes host strings");
        validate_host_strings(S, "S");
        const Key key(arch_name(), tau, length_bucket(mean_length(S)));

        int64_t ref_pairs = -1;
        int trials = 0;
        auto measure = [&](const TuneParams& p) {
            // best of two runs
            double best = 1e300;
            for (int r = 0; r < 2; ++r) {
                int64_t pairs = 0;
                best = std::min(best, time_one(S, tau, opt, p, &pairs));
                if (ref_pairs < 0) ref_pairs = pairs;
                if (pairs != ref_pairs)
                    throw Error(PJ_EDEVICE, "launch parameters changed the result (%lld vs %lld "
                                "pairs)", (long long)pairs, (long long)ref_pairs);
            }
            ++trials;
            return best;
        };
        TuneParams cur;
        (void)measure(cur);                  // warm-up: allocations, code objects, caches
        const double ms_default = measure(cur);
        double ms_best = ms_default;
        // measured settings, so a later pass does not time one again
        std::map<std::tuple<int, int, int, int, int, int>, double> seen;
        auto key_of = [](const TuneParams& p) {
            return std::make_tuple(p.verify_waves_per_cu, p.seg_chunk, p.big_list,
                                   p.probe_blocks_per_cu, p.lane_cands, p.probe_map);
        };
        seen[key_of(cur)] = ms_default;
        bool changed = false;
        auto descend = [&](int TuneParams::*field, const int* opts, size_t nopts) {
            for (size_t i = 0; i < nopts; ++i) {
                if (opts[i] == cur.*field) continue;
                TuneParams cand = cur;
                cand.*field = opts[i];
                const auto k = key_of(cand);
                const auto it = seen.find(k);
                const double ms = it != seen.end() ? it->second : (seen[k] = measure(cand));
                if (ms < ms_best) {
                    ms_best = ms;
                    cur = cand;
                    changed = true;
                }
            }
        };
        // coordinate descent, repeated until a whole pass changes nothing (at most 3 passes):
        // the parameters interact (e.g. the best lanes-per-candidate depends on the grid)
        for (int pass = 0; pass < 3; ++pass) {
            changed = false;
            descend(&TuneParams::big_list, kBigOpts, sizeof kBigOpts / sizeof kBigOpts[0]);
            descend(&TuneParams::seg_chunk, kChunkOpts, sizeof kChunkOpts / sizeof kChunkOpts[0]);
            descend(&TuneParams::verify_waves_per_cu, kWavesOpts,
                    sizeof kWavesOpts / sizeof kWavesOpts[0]);
            descend(&TuneParams::lane_cands, kLaneOpts, sizeof kLaneOpts / sizeof kLaneOpts[0]);
            descend(&TuneParams::probe_blocks_per_cu, kProbeOpts,
                    sizeof kProbeOpts / sizeof kProbeOpts[0]);
            descend(&TuneParams::probe_map, kMapOpts, sizeof kMapOpts / sizeof kMapOpts[0]);
            if (!changed) break;
        }

        {
            std::lock_guard<std::mutex> lk(g_mu);
            g_local[key] = Entry{cur, ms_best};
            if (opt && opt->tune_cache && opt->tune_cache[0]) {
                auto& t = file_table(opt->tune_cache);
                t[key] = Entry{cur, ms_best};
                write_file(opt->tune_cache, t);
                FileState& fs = g_files[opt->tune_cache];
                stat_file(opt->tune_cache, fs.mtime_ns, fs.size);
            }
        }
        out->verify_waves_per_cu = cur.verify_waves_per_cu;
        out->seg_chunk = cur.seg_chunk;
        out->big_list = cur.big_list;
        out->probe_blocks_per_cu = cur.probe_blocks_per_cu;
        out->lane_cands = cur.lane_cands;
        out->probe_map = cur.probe_map;
        out->len_bucket = std::get<2>(key);
        out->trials = trials;
        out->ms_default = ms_default;
        out->ms_best = ms_best;
        t_last_error.clear();
        return PJ_OK;
    } catch (const Error& e) {
        t_last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        t_last_error = "host allocation failed";
        return PJ_ENOMEM;
    }
}

}  // extern "C"

namespace pj {

static double time_one(const pj_strings* S, int32_t tau, const pj_options* base,
                       const TuneParams& p, int64_t* pairs)
{
    pj_options o{};
    if (base) o = *base;
    o.mode = PJ_MODE_BATCHED;
    o.outputs_on_device = 1;
    o.tune_cache = nullptr;
    pj_pairs out{};
    const int rc = self_join_with(S, tau, &o, &out, &p);
    if (rc != PJ_OK) throw Error(rc, "%s", t_last_error.c_str());
    *pairs = out.count;
    pj_pairs_free(&out);
    // the probe and verification phases (kernels plus the bucketing, scans and chunk set-up
    // between them, which the list-size threshold and the grids also change)
    const pj_stats& st = t_last_ok_stats;
    return st.ms_probe + st.ms_verify;
}

}  // namespace pj
