// Host-only check of the serving form's admission and deadline policy
// (paper_1611_09704_amd/csrc/spd_admit.h) with a fake clock and a fake
// executor: chunks "run" for a set time per beam and finish in admission
// order per beam.  Built and run by tests/test_serve_policy_cpu.py.
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "spd_admit.h"

struct Req {
    int beam;
    long seq;
    long arrival;        // arrival order
};

struct Running {
    int beam, buf;
    long seq;
    double done;
};

static int fails = 0;
#define CHECK(c, ...)                                    \
    do {                                                 \
        if (!(c)) {                                      \
            std::printf("FAIL %s:%d: ", __FILE__, __LINE__); \
            std::printf(__VA_ARGS__);                    \
            std::printf("\n");                           \
            ++fails;                                     \
        }                                                \
    } while (0)

// One scenario: n_beams beams, chunks per beam, pool buffers, slots per beam,
// per-beam run time, arrivals every `gap` time units in a shuffled beam order.
static void scenario(int n_beams, int chunks, int pool, int slots, double gap, unsigned seed)
{
    std::mt19937 rng(seed);
    std::vector<double> run(n_beams);
    for (auto& r : run) r = 0.5 + (rng() % 1000) / 250.0;
    // arrivals: each beam's chunks in order, beams interleaved at random
    std::vector<Req> arrivals;
    std::vector<long> next(n_beams, 0);
    for (long a = 0; a < (long)n_beams * chunks; ++a) {
        int b;
        do b = (int)(rng() % n_beams); while (next[b] >= chunks);
        arrivals.push_back({b, next[b]++, a});
    }
    std::deque<Req> pending;
    std::vector<int> free_bufs;
    for (int i = 0; i < pool; ++i) free_bufs.push_back(i);
    std::vector<int> on_device(n_beams, 0);
    std::vector<char> blocked;
    std::vector<Running> running;
    std::vector<long> last_admitted(n_beams, -1);
    std::set<int> bufs_in_use;
    double t = 0.0;
    size_t ai = 0;
    long admitted = 0, completed = 0;
    for (int guard = 0; guard < 1000000; ++guard) {
        // arrivals due by now
        while (ai < arrivals.size() && ai * gap <= t) pending.push_back(arrivals[ai++]);
        // one admission pass, then check that nothing admissible was skipped
        std::vector<Req> admitted_now;
        const int n = spd::admit_pending(pending, free_bufs, on_device, slots, blocked, [&](Req& r, int buf) {
            CHECK(!bufs_in_use.count(buf), "buffer %d handed out twice", buf);
            bufs_in_use.insert(buf);
            CHECK(r.seq == last_admitted[r.beam] + 1, "beam %d admitted chunk %ld after %ld", r.beam, r.seq,
                  last_admitted[r.beam]);
            last_admitted[r.beam] = r.seq;
            running.push_back({r.beam, buf, r.seq, t + run[r.beam]});
            admitted_now.push_back(r);
            return true;
        });
        CHECK(n == (int)admitted_now.size(), "admit count %d vs %zu", n, admitted_now.size());
        admitted += n;
        for (int b = 0; b < n_beams; ++b) CHECK(on_device[b] <= slots, "beam %d has %d > %d on device", b, on_device[b], slots);
        CHECK((int)bufs_in_use.size() <= pool, "%zu buffers in use > pool %d", bufs_in_use.size(), pool);
        if (!free_bufs.empty()) {
            // every request still pending is blocked: its beam is full or an earlier one of it waits
            std::vector<char> seen(n_beams, 0);
            for (const Req& r : pending) {
                CHECK(seen[r.beam] || on_device[r.beam] >= slots,
                      "request (beam %d, chunk %ld) left pending with a free buffer and room", r.beam, r.seq);
                seen[r.beam] = 1;
            }
        }
        if (running.empty() && pending.empty() && ai == arrivals.size()) break;
        // advance the clock to the next event: an arrival or the earliest completion
        double tn = ai < arrivals.size() ? ai * gap : 1e300;
        for (const Running& r : running) tn = r.done < tn ? r.done : tn;
        CHECK(tn < 1e299, "stalled at t=%g with %zu pending", t, pending.size());
        if (!(tn < 1e299)) break;
        t = tn;
        for (size_t i = 0; i < running.size();) {
            if (running[i].done <= t) {
                free_bufs.push_back(running[i].buf);
                bufs_in_use.erase(running[i].buf);
                --on_device[running[i].beam];
                ++completed;
                running.erase(running.begin() + (long)i);
            } else {
                ++i;
            }
        }
    }
    CHECK(admitted == (long)n_beams * chunks, "admitted %ld of %ld", admitted, (long)n_beams * chunks);
    CHECK(completed == admitted, "completed %ld of %ld", completed, admitted);
    for (int b = 0; b < n_beams; ++b) CHECK(last_admitted[b] == chunks - 1, "beam %d reached chunk %ld", b, last_admitted[b]);
}

int main()
{
    // ample buffers; fewer buffers than beams (backpressure); one slot per beam; bursts (gap 0)
    scenario(4, 20, 8, 2, 0.3, 1u);
    scenario(6, 15, 3, 2, 0.1, 2u);
    scenario(3, 30, 3, 1, 0.0, 3u);
    scenario(16, 8, 5, 3, 0.05, 4u);
    scenario(1, 50, 2, 2, 1.0, 5u);
    // a launch failure: the request is dropped, its buffer returns, the pass stops
    {
        std::deque<Req> pending{{0, 0, 0}, {1, 0, 1}, {2, 0, 2}};
        std::vector<int> free_bufs{0, 1, 2}, on_device{0, 0, 0};
        std::vector<char> blocked;
        std::vector<long> launched;
        const int n = spd::admit_pending(pending, free_bufs, on_device, 2, blocked, [&](Req& r, int) {
            launched.push_back(r.arrival);
            return r.arrival != 1;
        });
        CHECK(n == 1 && launched.size() == 2, "failure pass admitted %d, launched %zu", n, launched.size());
        CHECK(pending.size() == 1 && pending.front().beam == 2, "failure pass left %zu pending", pending.size());
        CHECK(free_bufs.size() == 2 && on_device[0] == 1 && on_device[1] == 0, "failure pass resources");
    }
    // deadlines
    CHECK(!spd::overdue(10.0, 9.0, 0.0), "no deadline");
    CHECK(!spd::overdue(10.0, 9.5, 1.0), "within deadline");
    CHECK(spd::overdue(10.0, 8.5, 1.0), "past deadline");
    if (fails) return 1;
    std::printf("ok\n");
    return 0;
}
