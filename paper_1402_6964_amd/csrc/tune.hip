// Autotune table of the TSQR launch geometry (host side).
//
// tsnmf_tune_load reads a text table written by the autotuner
// (paper_1402_6964_amd/tune.py); tsnmf_tsqr_r then applies the entry that
// matches each call.  A line
//     tsqr <f32|f64> <row|col> <leaf f32|f64> <ld == n: 1|0> <n> <floor(log2 m)> <leaf_rows> <tree_arity> [<wy_panel>]
// keys an entry by input dtype, layout, row-block precision, whether rows are
// contiguous, width and row-count bucket; a line
//     batch <shift class 0> <shift class 1> <shift class 2> <shift class 3>
// gives the slab doubling per width class of the batched call; '#' starts a
// comment.  Every entry changes only the launch geometry, so the result
// equals the default's up to rounding.
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "common.hpp"

namespace tsnmf {
namespace {

using Key = std::tuple<int, int, int, int, int, int>;   // dtype, col, leaf64, ldeq, n, log2 m
std::mutex g_tune_mu;
std::map<Key, tsnmf_tsqr_config> g_tune;
int g_batch_shift = 0;

int floor_log2(int64_t m) {
    int r = 0;
    while (m > 1) {
        m >>= 1;
        ++r;
    }
    return r;
}

Key key_of(uint32_t flags, int64_t m, int n, int64_t ld) {
    const int dt = (flags & TSNMF_DTYPE_MASK) == TSNMF_F64 ? 64 : 32;
    const int col = (flags & TSNMF_COL_MAJOR) ? 1 : 0;
    const int leaf64 = (dt == 64 || (flags & TSNMF_LEAF_F64)) ? 1 : 0;
    const int ldeq = (col ? ld == m : ld == n) ? 1 : 0;
    return Key{dt, col, leaf64, ldeq, n, floor_log2(m)};
}

}  // namespace

int tune_batch_shift() {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return g_batch_shift;
}

bool tune_lookup(uint32_t flags, int64_t m, int n, int64_t ld, tsnmf_tsqr_config* out) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (g_tune.empty()) return false;
    auto it = g_tune.find(key_of(flags, m, n, ld));
    if (it == g_tune.end()) return false;
    *out = it->second;
    return true;
}

}  // namespace tsnmf

using namespace tsnmf;

extern "C" int tsnmf_tune_load(const char* path) {
    if (path == nullptr) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune.clear();
        g_batch_shift = 0;
        return TSNMF_OK;
    }
    FILE* f = std::fopen(path, "r");
    if (f == nullptr) return -1;
    std::map<Key, tsnmf_tsqr_config> table;
    int batch_shift = 0;
    char line[512];
    bool ok = true;
    while (std::fgets(line, sizeof line, f) != nullptr) {
        char* hash = std::strchr(line, '#');
        if (hash != nullptr) *hash = '\0';
        int bs[4];
        char bkind[16];
        if (std::sscanf(line, "%15s", bkind) == 1 && !std::strcmp(bkind, "batch")) {
            if (std::sscanf(line, "%15s %d %d %d %d", bkind, &bs[0], &bs[1], &bs[2], &bs[3]) != 5) {
                ok = false;
                break;
            }
            batch_shift = 0;
            for (int c = 0; c < 4; ++c) {
                if (bs[c] < 0 || bs[c] > 8) ok = false;
                batch_shift |= (bs[c] & 0xff) << (8 * c);
            }
            if (!ok) break;
            continue;
        }
        char kind[16], dt[8], lay[8], leaf[8];
        int ldeq = 0, n = 0, lg = 0, arity = 0, wy = 0;
        long long leaf_rows = 0;
        const int got = std::sscanf(line, "%15s %7s %7s %7s %d %d %d %lld %d %d", kind, dt, lay, leaf, &ldeq, &n, &lg,
                                    &leaf_rows, &arity, &wy);
        if (got <= 0) continue;                          // blank or comment line
        const bool f32 = !std::strcmp(dt, "f32"), f64 = !std::strcmp(dt, "f64");
        const bool row = !std::strcmp(lay, "row"), col = !std::strcmp(lay, "col");
        const bool l32 = !std::strcmp(leaf, "f32"), l64 = !std::strcmp(leaf, "f64");
        if ((got != 9 && got != 10) || (wy != 0 && wy != 1 && wy != 16) || std::strcmp(kind, "tsqr") != 0 || !(f32 || f64) || !(row || col) || !(l32 || l64) ||
            (f64 && l32) || (ldeq != 0 && ldeq != 1) || n < 1 || n > TSNMF_MAX_N || lg < 0 || lg > 62 ||
            leaf_rows < 0 || (arity != 0 && (arity < 2 || arity > 64))) {
            ok = false;
            break;
        }
        tsnmf_tsqr_config c{};
        c.leaf_rows = leaf_rows;
        c.tree_arity = arity;
        c.rows_per_lane = 0;
        c.wy_panel = wy;
        c.reserved = 0;
        table[Key{f64 ? 64 : 32, col ? 1 : 0, l64 ? 1 : 0, ldeq, n, lg}] = c;
    }
    std::fclose(f);
    if (!ok) return -1;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.swap(table);
    g_batch_shift = batch_shift;
    return TSNMF_OK;
}
