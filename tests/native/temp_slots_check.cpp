// Host check of the rule that picks a cached temporary block
// (paper_1702_08159_amd/csrc/temp_slots.hpp, the header the runtime uses).
#include <cstdio>
#include <cstdlib>

#include "temp_slots.hpp"

namespace {

struct Slot {
    size_t bytes = 0;
    bool used = false;
    bool busy = false;
    int last = 0;  // stands for the stream of the last use
};

int failures = 0;

void expect(int got, int want, const char* what)
{
    if (got != want) {
        std::printf("FAIL %s: got %d, want %d\n", what, got, want);
        ++failures;
    }
}

}  // namespace

int main()
{
    using mck::pick_temp_slot;
    Slot s[4];
    // nothing used yet: the first block
    expect(pick_temp_slot(s, 4, 1, 100), 0, "fresh blocks");
    // block 0 used on stream 1 (200 B), block 1 on stream 2 (500 B)
    s[0] = {200, true, false, 1};
    s[1] = {500, true, false, 2};
    expect(pick_temp_slot(s, 4, 1, 150), 0, "same stream, large enough");
    expect(pick_temp_slot(s, 4, 1, 300), 2, "same stream too small: a never-used block first");
    expect(pick_temp_slot(s, 4, 2, 300), 1, "the other stream's own block");
    expect(pick_temp_slot(s, 4, 3, 10), 2, "a new stream takes a never-used block, not a wait");
    // every block used: same stream too small is grown before waiting on another stream
    s[2] = {100, true, false, 3};
    s[3] = {100, true, false, 3};
    expect(pick_temp_slot(s, 4, 1, 300), 0, "grow the stream's own block");
    expect(pick_temp_slot(s, 4, 4, 10), 0, "unknown stream: any free block (device-side wait)");
    // busy blocks are never taken
    s[0].busy = true;
    expect(pick_temp_slot(s, 4, 1, 150), 1, "own block busy: another (with a wait)");
    for (Slot& t : s)
        t.busy = true;
    expect(pick_temp_slot(s, 4, 1, 1), -1, "all busy");
    // a block just grown (used = false) counts as never used
    s[3] = {4096, false, false, 2};
    expect(pick_temp_slot(s, 4, 1, 4000), 3, "grown block");
    if (failures == 0)
        std::printf("temp slot checks passed\n");
    return failures == 0 ? EXIT_SUCCESS : EXIT_FAILURE;
}
