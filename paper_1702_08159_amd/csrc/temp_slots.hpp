// temp_slots.hpp -- which cached temporary block a call takes.  No HIP
// here: the runtime holds the blocks, their events and the mutex, so that
// this rule also builds and runs in a plain host test.
#pragma once

#include <cstddef>

namespace mck {

// S must have the members `size_t bytes`, `bool used` (an event marks the
// end of the last call that used the block), `bool busy` (taken by a call
// not yet finished on the host) and `last` (the stream of that last use,
// comparable with `stream`).  Returns the index of the block to take, or -1
// when every block is busy.  In order of preference:
//   0. last used on this stream and large enough: stream order alone
//      protects it, nothing to wait for or allocate;
//   1. never used (or just grown): nothing to wait for;
//   2. last used on this stream but too small: grown, no wait;
//   3. any free block: the stream waits (on the device) for its last use.
template <class S, class Stream>
int pick_temp_slot(const S* slots, int count, Stream stream, size_t bytes)
{
    for (int pass = 0; pass < 4; ++pass) {
        for (int k = 0; k < count; ++k) {
            const S& t = slots[k];
            if (t.busy)
                continue;
            const bool same = t.used && t.last == stream;
            if ((pass == 0 && same && t.bytes >= bytes) || (pass == 1 && !t.used) || (pass == 2 && same) ||
                pass == 3)
                return k;
        }
    }
    return -1;
}

}  // namespace mck
