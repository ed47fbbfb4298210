// spd_admit.h -- the serving form's admission and deadline policy, host
// code only (no HIP), shared by the server's worker thread and its host-side
// policy test.
//
// Requests wait in arrival order.  One is admitted when a pool buffer is free
// and its beam has fewer than `slots` chunks on the device.  A beam's
// requests are admitted in their order: once one of a beam's requests cannot
// go, its later ones wait too, while other beams' requests behind it may go
// (no beam blocks another).  A chunk on the device longer than the deadline
// (seconds from admission; 0 = none) is overdue.
#pragma once

#include <cstdint>
#include <deque>
#include <vector>

namespace spd {

// Admits from `pending` (each Req has an int member `beam`) in one pass.
// on_device[b]: chunks of beam b on the device; free_bufs: the pool's free
// buffers (one is popped per admission and passed to launch).  launch(req,
// buf) enqueues the chunk and returns false on failure: the pass stops, the
// buffer goes back to the pool and the request is dropped from `pending`
// (the caller records the fault).  Returns the number admitted.
template <class Req, class Launch>
int admit_pending(std::deque<Req>& pending, std::vector<int>& free_bufs, std::vector<int>& on_device, int slots,
                  std::vector<char>& blocked, Launch&& launch)
{
    int n = 0;
    blocked.assign(on_device.size(), 0);
    for (auto it = pending.begin(); it != pending.end() && !free_bufs.empty();) {
        const int b = it->beam;
        if (blocked[b] || on_device[b] >= slots) {
            blocked[b] = 1;
            ++it;
            continue;
        }
        Req r = *it;
        it = pending.erase(it);
        const int buf = free_bufs.back();
        free_bufs.pop_back();
        if (!launch(r, buf)) {
            free_bufs.push_back(buf);
            break;
        }
        ++on_device[b];
        ++n;
    }
    return n;
}

// A chunk admitted at start_s and not finished at now_s has missed its deadline.
inline bool overdue(double now_s, double start_s, double deadline_s)
{
    return deadline_s > 0.0 && now_s - start_s > deadline_s;
}

}  // namespace spd
