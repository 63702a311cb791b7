// Autotuner table: the block width and variant measured fastest for a
// shape (m, n) on this machine.  The paper leaves the choice between block
// sizes and algorithms to profiling on the hardware at hand, as self-tuning
// packages do (Conclusion); jevd_autotune (api.hip) measures the candidates
// on a caller's matrix and records the winner here, jacobi_evd consults the
// table when opts->block is 0 or opts->variant is JEVD_VAR_AUTO.
//
// The table is kept per process and mirrored to a text file, one line per
// shape: "m n block variant ms" (the last record of a shape wins).  The
// batched solve's records, one per size class, are lines "batch class
// waves ms": the workgroup size (wavefronts) measured fastest for the class
// by jevd_batch_autotune, which jevd_batch_create then uses.  The
// file is JEVD_TUNE_FILE if set, else $HOME/.cache/jevd_tune.txt, else
// nothing is persisted; jevd_tune_file() points it elsewhere.  Host code
// only: no device work.
#include <sys/stat.h>

#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/jevd.h"
#include "block.h"
#include "jevd_internal.h"

namespace jevd {
namespace {

struct TuneEntry {
    int m, n, block, variant;
    double ms;
};

// batched solve: the workgroup size measured fastest for a size class
struct BatchTuneEntry {
    int cls, waves;
    double ms;
};

std::mutex g_mu;
std::vector<TuneEntry> g_tab;
std::vector<BatchTuneEntry> g_btab;
std::string g_path;
bool g_loaded = false;

std::string default_path()
{
    if (const char *p = std::getenv("JEVD_TUNE_FILE")) return p;
    if (const char *h = std::getenv("HOME")) return std::string(h) + "/.cache/jevd_tune.txt";
    return std::string();
}

// A record: a block variant with a block width the shape admits, or the
// pointwise variant with block 0.
bool valid_entry(const TuneEntry &e)
{
    if (e.n < 2 || e.m < e.n || !(e.ms >= 0.0)) return false;
    if (e.variant == JEVD_VAR_POINTWISE) return e.block == 0;
    return (e.variant == JEVD_VAR_BLOCK_ORIENTED || e.variant == JEVD_VAR_FULL_BLOCK) &&
           block_shape_supported(e.m, e.n, e.block);
}

bool valid_batch_entry(const BatchTuneEntry &e)
{
    return e.cls >= 0 && e.cls < kBatchClasses && batch_waves_supported(e.waves) && e.ms >= 0.0;
}

void put_batch(const BatchTuneEntry &e)
{
    for (BatchTuneEntry &x : g_btab)
        if (x.cls == e.cls) {
            x = e;
            return;
        }
    g_btab.push_back(e);
}

void put(const TuneEntry &e)
{
    for (TuneEntry &x : g_tab)
        if (x.m == e.m && x.n == e.n) {
            x = e;
            return;
        }
    g_tab.push_back(e);
}

// Reads the file at g_path into the table (lines that do not parse are
// skipped).  Caller holds g_mu.
void load_locked()
{
    g_loaded = true;
    if (g_path.empty()) return;
    FILE *f = std::fopen(g_path.c_str(), "r");
    if (!f) return;
    TuneEntry e;
    BatchTuneEntry be;
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
        if (std::sscanf(line, "batch %d %d %lf", &be.cls, &be.waves, &be.ms) == 3) {
            if (valid_batch_entry(be)) put_batch(be);
        } else if (std::sscanf(line, "%d %d %d %d %lf", &e.m, &e.n, &e.block, &e.variant, &e.ms) ==
                       5 &&
                   valid_entry(e)) {
            put(e);
        }
    }
    std::fclose(f);
}

void ensure_loaded_locked()
{
    if (g_loaded) return;
    g_path = default_path();
    load_locked();
}

// Rewrites the file from the table (best effort; a missing directory is
// created one level deep).  Caller holds g_mu.
int save_locked()
{
    if (g_path.empty()) return JEVD_OK;
    const std::string tmp = g_path + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f && errno == ENOENT) {
        const size_t slash = g_path.rfind('/');
        if (slash != std::string::npos && slash > 0) {
            (void)::mkdir(g_path.substr(0, slash).c_str(), 0755);
            f = std::fopen(tmp.c_str(), "w");
        }
    }
    if (!f) return JEVD_EINVAL;
    for (const TuneEntry &e : g_tab)
        std::fprintf(f, "%d %d %d %d %.6f\n", e.m, e.n, e.block, e.variant, e.ms);
    for (const BatchTuneEntry &e : g_btab) std::fprintf(f, "batch %d %d %.6f\n", e.cls, e.waves, e.ms);
    std::fclose(f);
    if (std::rename(tmp.c_str(), g_path.c_str()) != 0) return JEVD_EINVAL;
    return JEVD_OK;
}

bool lookup_locked(int m, int n, TuneEntry *out)
{
    ensure_loaded_locked();
    for (const TuneEntry &e : g_tab)
        if (e.m == m && e.n == n) {
            *out = e;
            return true;
        }
    return false;
}

}  // namespace

int tuned_block_width(int m, int n)
{
    std::lock_guard<std::mutex> lk(g_mu);
    TuneEntry e;
    return (lookup_locked(m, n, &e) && e.block > 0) ? e.block : -1;
}

int tuned_batch_waves(int cls)
{
    std::lock_guard<std::mutex> lk(g_mu);
    ensure_loaded_locked();
    for (const BatchTuneEntry &e : g_btab)
        if (e.cls == cls) return e.waves;
    return -1;
}

int tuned_variant(int m, int n)
{
    std::lock_guard<std::mutex> lk(g_mu);
    TuneEntry e;
    return lookup_locked(m, n, &e) ? e.variant : -1;
}

}  // namespace jevd

using namespace jevd;

extern "C" {

int jevd_tune_file(const char *path)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_tab.clear();
    g_btab.clear();
    g_path = path ? std::string(path) : default_path();
    load_locked();
    return JEVD_OK;
}

int jevd_tune_lookup(int m, int n, int *block, int *variant, double *ms)
{
    std::lock_guard<std::mutex> lk(g_mu);
    TuneEntry e;
    if (!lookup_locked(m, n, &e)) return JEVD_EINVAL;
    if (block) *block = e.block;
    if (variant) *variant = e.variant;
    if (ms) *ms = e.ms;
    return JEVD_OK;
}

int jevd_tune_record(int m, int n, int block, int variant, double ms)
{
    const TuneEntry e{m, n, block, variant, ms};
    if (!valid_entry(e)) return JEVD_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    ensure_loaded_locked();
    put(e);
    return save_locked();
}

int jevd_batch_tune_lookup(int size_class, int *waves, double *ms)
{
    std::lock_guard<std::mutex> lk(g_mu);
    ensure_loaded_locked();
    for (const BatchTuneEntry &e : g_btab)
        if (e.cls == size_class) {
            if (waves) *waves = e.waves;
            if (ms) *ms = e.ms;
            return JEVD_OK;
        }
    return JEVD_EINVAL;
}

int jevd_batch_tune_record(int size_class, int waves, double ms)
{
    const BatchTuneEntry e{size_class, waves, ms};
    if (!valid_batch_entry(e)) return JEVD_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    ensure_loaded_locked();
    put_batch(e);
    return save_locked();
}

}  // extern "C"
