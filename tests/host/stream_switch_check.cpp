// Host check of ram::switch_stream (ram_stream.h) with a stand-in runtime that
// tracks, per stream, the set of context calls its next work is ordered after.
// A context call made on stream s must be ordered after every earlier call of
// the context (they share its scratch), unless a capture was involved.
#include "ram_stream.h"

#include <cstdio>
#include <set>
#include <vector>

namespace {

struct Sim {
    using stream_t = int;
    using event_t = int;
    std::vector<std::set<int>> stream_after;   // calls stream s's next work waits for
    std::vector<std::set<int>> event_marks;    // calls an event stands for
    std::vector<bool> cap;
    int records = 0, waits = 0;
    int fail_record = 0;
    explicit Sim(int n) : stream_after(n), event_marks(1), cap(n, false) {}
    bool capturing(int s) { return cap[s]; }
    int record(int ev, int s)
    {
        if (fail_record) return fail_record;
        ++records;
        event_marks[ev] = stream_after[s];
        return 0;
    }
    int wait(int s, int ev)
    {
        ++waits;
        stream_after[s].insert(event_marks[ev].begin(), event_marks[ev].end());
        return 0;
    }
    // one context call on stream s: returns the calls it is ordered after
    std::set<int> call(int s, int id)
    {
        std::set<int> before = stream_after[s];
        stream_after[s].insert(id);
        return before;
    }
};

int failures = 0;
#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            std::printf("FAIL line %d: %s\n", __LINE__, #c);              \
            ++failures;                                                   \
        }                                                                 \
    } while (0)

// A sequence of (stream) calls through switch_stream: each call must be
// ordered after every earlier one.
void run_sequence(const std::vector<int> &streams, int n_streams)
{
    Sim sim(n_streams);
    int cur = streams.empty() ? 0 : streams[0];
    for (size_t i = 0; i < streams.size(); ++i) {
        CHECK(ram::switch_stream(sim, cur, streams[i], 0) == 0);
        CHECK(cur == streams[i]);
        const std::set<int> before = sim.call(cur, (int)i);
        for (size_t j = 0; j < i; ++j) CHECK(before.count((int)j) == 1);
    }
}

}  // namespace

int main()
{
    // staying on one stream: no events at all
    {
        Sim sim(2);
        int cur = 0;
        for (int i = 0; i < 5; ++i) CHECK(ram::switch_stream(sim, cur, 0, 0) == 0);
        CHECK(sim.records == 0 && sim.waits == 0);
    }
    // one switch: one record on the old stream, one wait on the new one
    {
        Sim sim(2);
        int cur = 0;
        sim.call(0, 0);
        CHECK(ram::switch_stream(sim, cur, 1, 0) == 0);
        CHECK(cur == 1 && sim.records == 1 && sim.waits == 1);
        CHECK(sim.call(1, 1).count(0) == 1);
    }
    // back and forth, three streams, repeated visits, the null stream (0)
    run_sequence({0, 1, 0, 1, 1, 2, 0, 2, 1, 0}, 3);
    run_sequence({2, 2, 2, 1, 2, 0, 0, 1}, 3);
    // a capturing stream on either side: no hand-off, the switch still happens
    {
        Sim sim(2);
        int cur = 0;
        sim.cap[1] = true;
        CHECK(ram::switch_stream(sim, cur, 1, 0) == 0);
        CHECK(cur == 1 && sim.records == 0 && sim.waits == 0);
        CHECK(ram::switch_stream(sim, cur, 0, 0) == 0);
        CHECK(cur == 0 && sim.records == 0 && sim.waits == 0);
    }
    // a failing record: the error comes back and the context stays put
    {
        Sim sim(2);
        int cur = 0;
        sim.fail_record = 7;
        CHECK(ram::switch_stream(sim, cur, 1, 0) == 7);
        CHECK(cur == 0 && sim.waits == 0);
    }
    if (failures) {
        std::printf("%d failures\n", failures);
        return 1;
    }
    std::printf("stream hand-off: all checks passed\n");
    return 0;
}
