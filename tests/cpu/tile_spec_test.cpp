// CPU check of the stream tile choice's host logic (tile_spec.h): cache
// lines, the FJOFC_TILE override and the pick of a cache row.  Prints
// "N failures".
#include "tile_spec.h"

#include <cstdio>

using namespace fjofc;

static int failures = 0;
#define CHECK(cond)                                                   \
    do {                                                              \
        if (!(cond)) {                                                \
            std::printf("FAIL line %d: %s\n", __LINE__, #cond);       \
            ++failures;                                               \
        }                                                             \
    } while (0)

static bool valid(int th, int var) { return th >= 8 && th <= 2048 && th % 8 == 0 && var >= 0 && var < 6; }

int main() {
    TuneRow r;
    CHECK(parse_tune_line("gfx950 5 1073741824 384 4   # m=3 n=20000: 517.5 us\n", valid, r));
    CHECK(r.arch == "gfx950" && r.d == 5 && r.nmax == 1073741824 && r.th == 384 && r.variant == 4);
    CHECK(!parse_tune_line("# arch d n_max tile_height variant\n", valid, r));
    CHECK(!parse_tune_line("   # indented comment\n", valid, r));
    CHECK(!parse_tune_line("gfx950 5 4096 100 4\n", valid, r));   // height not a multiple of 8
    CHECK(!parse_tune_line("gfx950 5 4096 128 6\n", valid, r));   // no variant 6
    CHECK(!parse_tune_line("gfx950 0 4096 128 1\n", valid, r));   // d < 1
    CHECK(!parse_tune_line("gfx950 5 4096 128\n", valid, r));     // a field missing
    CHECK(!parse_tune_line("", valid, r));

    int th = -1, var = -1;
    CHECK(!parse_tile_override(nullptr, 100, 2, valid, th, var));
    CHECK(!parse_tile_override("", 100, 2, valid, th, var));
    CHECK(parse_tile_override("64:1", 100, 2, valid, th, var) && th == 64 && var == 1);
    CHECK(!parse_tile_override("63:1", 100, 2, valid, th, var));
    CHECK(!parse_tile_override("64:1x", 100, 2, valid, th, var));
    const char *sc = "2:100:220:96:4,5:10000:30000:128:1,2:221:400:256:5";
    CHECK(parse_tile_override(sc, 200, 2, valid, th, var) && th == 96 && var == 4);
    CHECK(parse_tile_override(sc, 100, 2, valid, th, var) && th == 96 && var == 4);
    CHECK(parse_tile_override(sc, 220, 2, valid, th, var) && th == 96 && var == 4);
    CHECK(parse_tile_override(sc, 221, 2, valid, th, var) && th == 256 && var == 5);
    CHECK(!parse_tile_override(sc, 401, 2, valid, th, var));
    CHECK(!parse_tile_override(sc, 200, 3, valid, th, var));
    CHECK(parse_tile_override(sc, 20000, 5, valid, th, var) && th == 128 && var == 1);
    CHECK(parse_tile_override("bad,2:1:50:64:2", 40, 2, valid, th, var) && th == 64 && var == 2);
    CHECK(parse_tile_override("2:1:50:63:2,96:5", 40, 2, valid, th, var) && th == 96 && var == 5);

    std::vector<TuneRow> rows = {
        {"gfx950", 2, 128, 96, 1}, {"gfx950", 2, 256, 128, 5}, {"gfx950", 2, 1073741824, 384, 5},
        {"gfx950", 5, 2048, 128, 5}, {"gfx950", 5, 1073741824, 384, 4},
        {"gfx000", 3, 1073741824, 512, 3},
    };
    CHECK(pick_tune_row(rows, "gfx950", 100, 2, th, var) && th == 96 && var == 1);
    CHECK(pick_tune_row(rows, "gfx950", 128, 2, th, var) && th == 96 && var == 1);
    CHECK(pick_tune_row(rows, "gfx950", 129, 2, th, var) && th == 128 && var == 5);
    CHECK(pick_tune_row(rows, "gfx950", 5000, 2, th, var) && th == 384 && var == 5);
    // no d = 3 rows on this arch: nearest d, the larger on a tie (2 and 5
    // are 1 and 2 away: 2); the other arch's d = 3 row is ignored
    CHECK(pick_tune_row(rows, "gfx950", 1000, 3, th, var) && th == 384 && var == 5);
    // d = 4: 5 is nearer than 2
    CHECK(pick_tune_row(rows, "gfx950", 1000, 4, th, var) && th == 128 && var == 5);
    CHECK(pick_tune_row(rows, "gfx950", 20000, 8, th, var) && th == 384 && var == 4);
    CHECK(pick_tune_row(rows, "gfx950", 1000, 1, th, var) && th == 384 && var == 5);
    th = var = -7;
    CHECK(!pick_tune_row(rows, "gfx942", 1000, 5, th, var) && th == -7 && var == -7);
    std::vector<TuneRow> capped = {{"gfx950", 2, 256, 64, 1}};
    CHECK(!pick_tune_row(capped, "gfx950", 257, 2, th, var));

    std::printf("%d failures\n", failures);
    return failures ? 1 : 0;
}
