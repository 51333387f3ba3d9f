// Autotune cache file of the batched evaluation (host code only).
//
// A text file of one line per tuned batch,
//   <key> TAB <depth of every box, comma-separated> TAB <P2P groups, same> LF
// where the key names what the timings depend on: the device architecture,
// the order, the precision mode, the FP64 top levels and every box's edge and
// atom count.  Lines are only appended, each with one write; the last valid
// line for a key wins, and lines that do not parse (a torn or foreign line)
// are skipped.
#include <algorithm>
#include <cstdio>
#include <string>
#include <vector>

#include "fmm_internal.h"

namespace fmm {

std::string tuning_cache_key(const std::string &arch, int p, int prec, int fp64_levels, size_t nbox,
                             const double *box, const int64_t *natoms) {
    std::string a = arch.empty() ? "unknown" : arch;
    for (char &c : a)
        if (c == '\t' || c == '\n' || c == '\r' || c == ' ') c = '_';
    char buf[96];
    std::snprintf(buf, sizeof buf, " p=%d prec=%d fp64_levels=%d boxes=", p, prec, fp64_levels);
    std::string key = "fmm-autotune-1 arch=" + a + buf;
    for (size_t w = 0; w < nbox; ++w) {
        std::snprintf(buf, sizeof buf, "%s%.17g:%lld", w ? "," : "", box[w], (long long)natoms[w]);
        key += buf;
    }
    return key;
}

// exactly nbox comma-separated decimal ints in f
static bool parse_ints(const std::string &f, size_t nbox, std::vector<int> &out) {
    out.clear();
    size_t i = 0;
    while (i <= f.size() && out.size() < nbox) {
        const size_t j = std::min(f.find(',', i), f.size());
        if (j == i) return false;
        int v = 0;
        for (size_t k = i; k < j; ++k) {
            if (f[k] < '0' || f[k] > '9' || v > 100000) return false;
            v = 10 * v + (f[k] - '0');
        }
        out.push_back(v);
        i = j + 1;
    }
    return out.size() == nbox && i == f.size() + 1;
}

bool tuning_cache_lookup(const char *path, const std::string &key, size_t nbox, std::vector<int> &levels,
                         std::vector<int> &groups) {
    FILE *fp = std::fopen(path, "rb");
    if (!fp) return false;
    bool hit = false;
    std::string line;
    std::vector<int> lv, gr;
    auto take = [&]() {
        const size_t t1 = line.find('\t');
        if (t1 != key.size() || line.compare(0, t1, key) != 0) return;
        const size_t t2 = line.find('\t', t1 + 1);
        if (t2 == std::string::npos) return;
        if (!parse_ints(line.substr(t1 + 1, t2 - t1 - 1), nbox, lv) || !parse_ints(line.substr(t2 + 1), nbox, gr))
            return;
        for (size_t w = 0; w < nbox; ++w)
            if (lv[w] < 1 || lv[w] > kMaxLevels || !valid_p2p_groups(gr[w])) return;
        levels = lv;
        groups = gr;
        hit = true;
    };
    int c;
    while ((c = std::fgetc(fp)) != EOF) {
        if (c == '\n') {
            take();
            line.clear();
        } else {
            line.push_back((char)c);
        }
    }
    // a last line without its line feed is a torn append: skipped
    std::fclose(fp);
    return hit;
}

bool tuning_cache_append(const char *path, const std::string &key, const std::vector<int> &levels,
                         const std::vector<int> &groups) {
    std::string line = key + "\t";
    for (size_t w = 0; w < levels.size(); ++w) line += (w ? "," : "") + std::to_string(levels[w]);
    line += "\t";
    for (size_t w = 0; w < groups.size(); ++w) line += (w ? "," : "") + std::to_string(groups[w]);
    line += "\n";
    FILE *fp = std::fopen(path, "ab");
    if (!fp) return false;
    const bool ok = std::fwrite(line.data(), 1, line.size(), fp) == line.size();
    return std::fclose(fp) == 0 && ok;
}

}  // namespace fmm
