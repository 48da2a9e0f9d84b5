// Persisted autotune results of the batch engine (declared in include/rz.h,
// "autotune cache") and the point-order classifier of its key.  Host code
// only: the batch engine copies its samples to the host before calling it.
//
// Cache file: plain text, one entry per line,
//   <arch> n<log2 points> px<log2 pixels> v<views> hq<eighths> <order> k=.. \
//       block=.. ppt=.. early_out=.. xcd=.. bin=.. hq_block=.. hq_ppt=.. \
//       hq_early_out=.. hq_xcd=.. hq_bin=.. ms=..
// The first six words are the key.  Lines starting with '#' and lines that
// do not parse are ignored (and dropped when the file is rewritten).
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#include <algorithm>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "rz.h"

namespace rz {
namespace {

constexpr int kKeyWords = 6;
constexpr int64_t kWindow = 4096;

std::mutex g_cache_mu;   // one writer at a time inside a process

bool valid_launch(const rz_launch &l)
{
    return (l.block == 64 || l.block == 128 || l.block == 256 || l.block == 512) &&
           (l.ppt == 4 || l.ppt == 8 || l.ppt == 16) && (l.early_out & ~1) == 0 &&
           (l.xcd_remap & ~1) == 0 && l.bin >= 0 && l.bin <= 3;
}

bool valid_entry(const rz_tune_entry &e)
{
    return e.views_per_group >= 1 && e.views_per_group <= 8 && valid_launch(e.depth) &&
           valid_launch(e.accum) && isfinite(e.ms) && e.ms >= 0.f;
}

// A key is six words of printable characters without spaces.
bool valid_key(const char *key)
{
    if (!key)
        return false;
    int words = 0;
    bool in_word = false;
    for (const char *c = key; *c; ++c) {
        if (*c == ' ') {
            if (!in_word)
                return false;   // leading or double space
            in_word = false;
        } else if (*c > ' ' && *c < 127) {
            if (!in_word)
                ++words;
            in_word = true;
        } else {
            return false;
        }
    }
    return in_word && words == kKeyWords;
}

// Splits a line into its key (first six words) and the rest.
bool split_line(const std::string &line, std::string *key, std::string *rest)
{
    std::istringstream in(line);
    std::string w, k;
    for (int i = 0; i < kKeyWords; ++i) {
        if (!(in >> w))
            return false;
        k += (i ? " " : "") + w;
    }
    *key = k;
    std::getline(in, *rest);
    return true;
}

bool parse_values(const std::string &rest, rz_tune_entry *e)
{
    struct Field {
        const char *name;
        int32_t *i;
    } fields[] = {
        {"k", &e->views_per_group},       {"block", &e->depth.block},
        {"ppt", &e->depth.ppt},           {"early_out", &e->depth.early_out},
        {"xcd", &e->depth.xcd_remap},     {"bin", &e->depth.bin},
        {"hq_block", &e->accum.block},    {"hq_ppt", &e->accum.ppt},
        {"hq_early_out", &e->accum.early_out}, {"hq_xcd", &e->accum.xcd_remap},
        {"hq_bin", &e->accum.bin},
    };
    const int nf = (int)(sizeof(fields) / sizeof(fields[0]));
    bool seen[16] = {};
    bool seen_ms = false;
    std::istringstream in(rest);
    std::string tok;
    while (in >> tok) {
        const size_t eq = tok.find('=');
        if (eq == std::string::npos)
            return false;
        const std::string name = tok.substr(0, eq), val = tok.substr(eq + 1);
        char *end = nullptr;
        if (name == "ms") {
            const double v = strtod(val.c_str(), &end);
            if (end == val.c_str() || *end)
                return false;
            e->ms = (float)v;
            seen_ms = true;
            continue;
        }
        int f = 0;
        while (f < nf && name != fields[f].name)
            ++f;
        if (f == nf)
            return false;
        const long v = strtol(val.c_str(), &end, 10);
        if (end == val.c_str() || *end || v < -1000000 || v > 1000000)
            return false;
        *fields[f].i = (int32_t)v;
        seen[f] = true;
    }
    for (int f = 0; f < nf; ++f)
        if (!seen[f])
            return false;
    return seen_ms && valid_entry(*e);
}

std::string format_line(const char *key, const rz_tune_entry &e)
{
    char buf[512];
    snprintf(buf, sizeof(buf),
             "%s k=%d block=%d ppt=%d early_out=%d xcd=%d bin=%d hq_block=%d hq_ppt=%d "
             "hq_early_out=%d hq_xcd=%d hq_bin=%d ms=%.4f",
             key, e.views_per_group, e.depth.block, e.depth.ppt, e.depth.early_out,
             e.depth.xcd_remap, e.depth.bin, e.accum.block, e.accum.ppt, e.accum.early_out,
             e.accum.xcd_remap, e.accum.bin, (double)e.ms);
    return buf;
}

// Median distance between consecutive points of x[i0 .. i0+m) against the
// diagonal of their bounding box: true when the window is spatially ordered.
// Returns false with *usable = false when fewer than 16 finite pairs exist.
bool window_ordered(const float *x, const float *y, const float *z, int64_t m, bool *usable)
{
    std::vector<double> d;
    d.reserve((size_t)m);
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = 0; i < m; ++i) {
        const double p[3] = {x[i], y[i], z[i]};
        if (!isfinite(p[0]) || !isfinite(p[1]) || !isfinite(p[2]))
            continue;
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], p[a]);
            hi[a] = std::max(hi[a], p[a]);
        }
        if (i > 0 && isfinite(x[i - 1]) && isfinite(y[i - 1]) && isfinite(z[i - 1])) {
            const double dx = p[0] - x[i - 1], dy = p[1] - y[i - 1], dz = p[2] - z[i - 1];
            d.push_back(sqrt(dx * dx + dy * dy + dz * dz));
        }
    }
    *usable = d.size() >= 16;
    if (!*usable)
        return false;
    std::nth_element(d.begin(), d.begin() + d.size() / 2, d.end());
    const double med = d[d.size() / 2];
    const double ex = hi[0] - lo[0], ey = hi[1] - lo[1], ez = hi[2] - lo[2];
    const double diag = sqrt(ex * ex + ey * ey + ez * ez);
    return med * 16.0 <= diag;   // consecutive points lie close together
}

}  // namespace

// Order class of host-resident points: windows of up to 4096 consecutive
// points at the start, middle and end; the majority of usable windows
// decides (ties: shuffled).  0 ordered, 1 shuffled.
int order_class(const float *x, const float *y, const float *z, int64_t n)
{
    const int64_t m = std::min(n, kWindow);
    const int64_t starts[3] = {0, (n - m) / 2, n - m};
    int ordered = 0, usable = 0;
    for (int w = 0; w < 3; ++w) {
        bool ok = false;
        const bool o = window_ordered(x + starts[w], y + starts[w], z + starts[w], m, &ok);
        usable += ok;
        ordered += ok && o;
    }
    return (usable > 0 && 2 * ordered > usable) ? 0 : 1;
}

int64_t order_sample_window() { return kWindow; }

// The same decision over windows already gathered on the host: window w is
// [w * m, (w + 1) * m) of each array.
int order_class_windows(const float *x, const float *y, const float *z, int64_t m, int nwin)
{
    int ordered = 0, usable = 0;
    for (int w = 0; w < nwin; ++w) {
        bool ok = false;
        const bool o = window_ordered(x + w * m, y + w * m, z + w * m, m, &ok);
        usable += ok;
        ordered += ok && o;
    }
    return (usable > 0 && 2 * ordered > usable) ? 0 : 1;
}

}  // namespace rz

extern "C" {

int rz_order_class_host(const float *x, const float *y, const float *z, int64_t n)
{
    if (n < 0 || (n > 0 && (!x || !y || !z)))
        return RZ_EINVAL;
    return rz::order_class(x, y, z, n);
}

int rz_tune_cache_lookup(const char *path, const char *key, rz_tune_entry *out)
{
    if (!path || !out || !rz::valid_key(key))
        return RZ_EINVAL;
    std::lock_guard<std::mutex> lock(rz::g_cache_mu);
    std::ifstream in(path);
    if (!in)
        return 0;   // no cache yet
    std::string line, k, rest;
    int found = 0;
    while (std::getline(in, line)) {
        if (line.empty() || line[0] == '#' || !rz::split_line(line, &k, &rest) || k != key)
            continue;
        rz_tune_entry e;
        memset(&e, 0, sizeof(e));
        if (rz::parse_values(rest, &e)) {
            *out = e;   // the last valid line of a key wins
            found = 1;
        }
    }
    return found;
}

int rz_tune_cache_store(const char *path, const char *key, const rz_tune_entry *entry)
{
    if (!path || !entry || !rz::valid_key(key) || !rz::valid_entry(*entry))
        return RZ_EINVAL;
    std::lock_guard<std::mutex> lock(rz::g_cache_mu);
    std::vector<std::string> keep;
    {
        std::ifstream in(path);
        std::string line, k, rest;
        while (in && std::getline(in, line)) {
            rz_tune_entry e;
            memset(&e, 0, sizeof(e));
            if (line.empty() || line[0] == '#' || !rz::split_line(line, &k, &rest) || k == key ||
                !rz::parse_values(rest, &e))
                continue;
            keep.push_back(line);
        }
    }
    keep.push_back(rz::format_line(key, *entry));
    // write a private temporary file, then rename it over the cache: a
    // reader sees the old file or the new one, never a torn one
    std::ostringstream tmpname;
    tmpname << path << ".tmp." << getpid() << "."
            << std::hash<std::thread::id>()(std::this_thread::get_id());
    const std::string tmp = tmpname.str();
    {
        std::ofstream out(tmp, std::ios::trunc);
        if (!out)
            return RZ_EIO;
        out << "# rz batch autotune cache: arch, log2 points, log2 pixels, views, splatting "
               "views in eighths, point order -> options\n";
        for (const std::string &l : keep)
            out << l << "\n";
        out.flush();
        if (!out) {
            out.close();
            unlink(tmp.c_str());
            return RZ_EIO;
        }
    }
    if (rename(tmp.c_str(), path) != 0) {
        unlink(tmp.c_str());
        return RZ_EIO;
    }
    return RZ_OK;
}

}  // extern "C"
