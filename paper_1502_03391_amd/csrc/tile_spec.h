// Host-only logic of the stream tile choice (no HIP): parsing the tile
// cache rows and the FJOFC_TILE override, and picking a cache row for a
// problem.  Kept free of device code so that it is also tested on the CPU.
#pragma once

#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

namespace fjofc {

struct TuneRow {
    std::string arch;
    int d, nmax, th, variant;
};

// One cache line "arch d n_max tile_height variant" ('#' starts a comment,
// also after the fields).  valid(th, variant) says whether the library has
// that tile.  Returns whether the line holds a usable row.
template <class Valid>
bool parse_tune_line(const char *line, Valid valid, TuneRow &r) {
    if (!line || line[0] == '#') return false;
    char arch[64];
    int d = 0, nmax = 0, th = 0, var = 0;
    if (std::sscanf(line, "%63s %d %d %d %d", arch, &d, &nmax, &th, &var) != 5) return false;
    if (arch[0] == '#' || d < 1 || nmax < 2 || !valid(th, var)) return false;
    r = TuneRow{arch, d, nmax, th, var};
    return true;
}

// FJOFC_TILE: "th:variant" for every problem, or a comma-separated list of
// "d:n_lo:n_hi:th:variant" entries, each for the problems of that d with
// n_lo <= n <= n_hi (the first matching entry applies).  Malformed or
// invalid entries are skipped.  Returns whether it set th and variant.
template <class Valid>
bool parse_tile_override(const char *spec, int n, int d, Valid valid, int &th, int &variant) {
    if (!spec || !*spec) return false;
    const std::string list(spec);
    size_t pos = 0;
    while (pos <= list.size()) {
        size_t end = list.find(',', pos);
        if (end == std::string::npos) end = list.size();
        const std::string it = list.substr(pos, end - pos);
        pos = end + 1;
        // an entry counts only if its fields use it up entirely
        int f[5], used = -1;
        const int len = (int)it.size();
        if (std::sscanf(it.c_str(), "%d:%d%n", &f[0], &f[1], &used) == 2 && used == len &&
            valid(f[0], f[1])) {
            th = f[0];
            variant = f[1];
            return true;
        }
        used = -1;
        if (std::sscanf(it.c_str(), "%d:%d:%d:%d:%d%n", &f[0], &f[1], &f[2], &f[3], &f[4],
                        &used) == 5 &&
            used == len && f[0] == d && f[1] <= n && n <= f[2] && valid(f[3], f[4])) {
            th = f[3];
            variant = f[4];
            return true;
        }
    }
    return false;
}

// The cache row for an (n, d) problem on arch: among the rows of arch, those
// of d, else of the nearest tabulated d (the larger one on a tie; a nearby
// d has a similar register footprint); of those, the smallest n_max >= n.
// Returns whether a row applies.
inline bool pick_tune_row(const std::vector<TuneRow> &rows, const std::string &arch, int n, int d,
                          int &th, int &variant) {
    int dt = -1;
    for (const TuneRow &r : rows) {
        if (r.arch != arch) continue;
        const int e = std::abs(r.d - d), et = std::abs(dt - d);
        if (dt < 0 || e < et || (e == et && r.d > dt)) dt = r.d;
    }
    int best = -1;
    for (const TuneRow &r : rows)
        if (r.arch == arch && r.d == dt && n <= r.nmax && (best < 0 || r.nmax < best)) {
            best = r.nmax;
            th = r.th;
            variant = r.variant;
        }
    return best >= 0;
}

}  // namespace fjofc
