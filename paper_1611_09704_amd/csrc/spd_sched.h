// spd_sched.h -- the host rule that decides whether a batched-run schedule
// read from the tuning cache can run a given plan.  Plain C++ (no HIP types),
// so the rule is also compiled and checked on its own on the host.
#pragma once

#include <stdint.h>

namespace spd {

// A cached schedule (outputs per lane X, register-window form `win`,
// persistent work-groups per CU, tiles per queue grab) is usable for a plan
// whose layout for that schedule has `tiles` tiles of `waves` waves when its
// fields are in range, the register-window form exists for the plan
// (has_win) and is asked for as a grid launch, and a grid launch
// (wgs_per_cu == 0, one work-group per tile) holds every tile in one launch of
// at most max_items work-items.  The cache key does not include the beam
// shapes, so the last test is what keeps a grid schedule tuned on small beams
// from being used for beams too large for one launch.
inline bool schedule_usable(int X, int win, int wgs_per_cu, int grab, bool has_win, int64_t tiles, int waves,
                            uint64_t max_items)
{
    if (!(X == 4 || X == 8) || wgs_per_cu < 0 || grab < 1 || waves < 1 || tiles < 0) return false;
    if (win && !(has_win && X == 8 && wgs_per_cu == 0)) return false;
    if (wgs_per_cu == 0 && (uint64_t)tiles * 64u * (uint64_t)waves > max_items) return false;
    return true;
}

}  // namespace spd
