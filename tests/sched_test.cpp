// CPU test of the request loop's admission logic (arena + FIFO admission + rounds).
// Built with g++ by tests/test_sched_cpu.py; prints one line per check, exits non-zero on
// the first failure.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <map>
#include <random>
#include <vector>

#include "ssvb_sched.h"

using ssvb::Admission;
using ssvb::Arena;

static int g_checks = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        ++g_checks;                                                           \
        if (!(c)) {                                                           \
            fprintf(stderr, "FAILED %s:%d: %s\n", __FILE__, __LINE__, #c);    \
            exit(1);                                                          \
        }                                                                     \
    } while (0)

static void arena_basics() {
    Arena a(1024, 64);
    uint64_t o1, o2, o3, o4;
    CHECK(a.alloc(100, &o1) && o1 == 0);    // 128 bytes
    CHECK(a.alloc(64, &o2) && o2 == 128);
    CHECK(a.alloc(500, &o3) && o3 == 192);  // 512 bytes
    CHECK(a.in_use() == 128 + 64 + 512 && a.check());
    CHECK(!a.alloc(400, &o4));              // 320 left
    CHECK(a.alloc(320, &o4) && o4 == 704 && a.in_use() == 1024 && a.check());
    CHECK(!a.alloc(1, &o4));
    a.release(o2, 64);                      // hole [128, 192)
    CHECK(a.check() && a.free_blocks() == 1 && a.largest_free() == 64);
    a.release(o1, 100);                     // merges with the hole after it: [0, 192)
    CHECK(a.check() && a.free_blocks() == 1 && a.largest_free() == 192);
    a.release(o4, 320);                     // [704, 1024) separate
    CHECK(a.check() && a.free_blocks() == 2);
    a.release(o3, 500);                     // everything merges
    CHECK(a.check() && a.free_blocks() == 1 && a.largest_free() == 1024 && a.in_use() == 0);
    CHECK(a.peak() == 1024);
    // first fit takes the lowest block that is large enough
    Arena b(1000, 1);
    uint64_t x[4];
    for (int i = 0; i < 4; ++i) CHECK(b.alloc(250, &x[i]) && x[i] == (uint64_t)(250 * i));
    b.release(x[0], 250);
    b.release(x[2], 250);
    uint64_t y;
    CHECK(b.alloc(200, &y) && y == 0);
    CHECK(b.alloc(100, &y) && y == 500);
    CHECK(b.check());
    // zero-byte requests take one aligned unit
    Arena c(256, 256);
    CHECK(c.alloc(0, &y) && y == 0 && c.in_use() == 256);
    printf("arena basics ok\n");
}

static void arena_random() {
    std::mt19937_64 rng(12345);
    for (uint64_t align : {1ull, 64ull, 256ull}) {
        Arena a(1 << 20, align);
        std::map<uint64_t, uint64_t> live;  // offset -> requested bytes
        uint64_t used = 0;
        for (int it = 0; it < 20000; ++it) {
            if (live.empty() || (rng() % 100) < 55) {
                const uint64_t n = 1 + rng() % 40000;
                uint64_t off;
                const bool ok = a.alloc(n, &off);
                if (!ok) {
                    CHECK(a.largest_free() < a.round_up(n));
                    continue;
                }
                CHECK(off % align == 0 && off + a.round_up(n) <= a.size());
                // no overlap with the live neighbours
                auto nx = live.lower_bound(off);
                if (nx != live.end()) CHECK(off + a.round_up(n) <= nx->first);
                if (nx != live.begin()) {
                    auto pv = std::prev(nx);
                    CHECK(pv->first + a.round_up(pv->second) <= off);
                }
                live[off] = n;
                used += a.round_up(n);
            } else {
                auto itl = live.begin();
                std::advance(itl, rng() % live.size());
                a.release(itl->first, itl->second);
                used -= a.round_up(itl->second);
                live.erase(itl);
            }
            CHECK(a.in_use() == used);
            if (it % 97 == 0) CHECK(a.check());
        }
        for (auto& l : live) a.release(l.first, l.second);
        CHECK(a.check() && a.in_use() == 0 && a.free_blocks() == 1 && a.largest_free() == a.size());
    }
    printf("arena random ok\n");
}

static void admission_fifo() {
    Admission q(1000, 64, 1);
    q.submit(1, 600);
    q.submit(2, 300);
    q.submit(3, 200);  // does not fit after 1 and 2 ...
    q.submit(4, 100);  // ... and 4, which would fit, may not overtake it
    std::vector<std::pair<uint64_t, uint64_t>> ad;
    CHECK(q.admit(ad) == 2 && ad[0].first == 1 && ad[1].first == 2 && ad[0].second == 0 && ad[1].second == 600);
    CHECK(q.queued() == 2 && q.ready() == 2 && q.resident() == 2);
    std::vector<uint64_t> r;
    CHECK(q.take_round(r) == 2 && r[0] == 1 && r[1] == 2);
    CHECK(q.ready() == 0);
    ad.clear();
    CHECK(q.admit(ad) == 0);  // nothing freed yet
    CHECK(q.finish(1) && !q.finish(1));
    CHECK(q.admit(ad) == 2 && ad[0].first == 3 && ad[1].first == 4);
    CHECK(q.arena().in_use() == 600 && q.arena().check());
    CHECK(q.fits_at_all(1000) && !q.fits_at_all(1001));
    printf("admission fifo ok\n");
}

static void admission_rounds_and_cancel() {
    Admission q(1 << 20, 3, 256);
    for (uint64_t t = 1; t <= 7; ++t) q.submit(t, 1000);
    std::vector<std::pair<uint64_t, uint64_t>> ad;
    CHECK(q.admit(ad) == 7);
    std::vector<uint64_t> r1, r2, r3;
    CHECK(q.take_round(r1) == 3 && q.take_round(r2) == 3 && q.take_round(r3) == 1);
    CHECK(r1[0] == 1 && r2[0] == 4 && r3[0] == 7);
    // cancel: ready requests free their memory, queued ones just leave the queue
    Admission c(4096, 64, 256);
    c.submit(1, 2000);
    c.submit(2, 2000);
    c.submit(3, 2000);
    ad.clear();
    CHECK(c.admit(ad) == 2);
    auto cr = c.cancel_ready();
    CHECK(cr.size() == 2 && c.arena().in_use() == 0 && c.resident() == 0);
    auto cq = c.cancel_queued();
    CHECK(cq.size() == 1 && cq[0] == 3 && c.queued() == 0);
    printf("admission rounds and cancel ok\n");
}

// Discrete-event run of the request loop's policy with a fake executor: each tick the
// loop retires rounds whose service time has elapsed, admits while memory allows, and
// starts one round per idle stream; a round takes the sum of its frames' costs.
static void policy_simulation() {
    std::mt19937_64 rng(7);
    const int streams = 2;
    Admission q(64ull << 20, 64, 256);
    struct Req {
        uint64_t bytes, cost, arrive, admit = 0, done = 0;
    };
    std::vector<Req> reqs(2000);
    uint64_t t = 0;
    for (auto& r : reqs) {
        t += rng() % 40;
        r.arrive = t;
        r.bytes = (1 + rng() % 16) << 20;  // 1..16 MiB
        r.cost = 10 + rng() % 200;
    }
    struct Round {
        bool busy = false;
        uint64_t end = 0;
        std::vector<uint64_t> tk;
    } rounds[streams];
    size_t next = 0, finished = 0;
    uint64_t admitted_order = 0, max_running = 0, overlapped = 0;
    for (uint64_t now = 0; finished < reqs.size(); ++now) {
        int running = 0;
        for (auto& R : rounds) {
            if (!R.busy) continue;
            if (R.end <= now) {
                for (uint64_t k : R.tk) {
                    CHECK(q.finish(k));
                    reqs[k - 1].done = now;
                    ++finished;
                }
                R.busy = false;
                R.tk.clear();
            } else {
                ++running;
            }
        }
        while (next < reqs.size() && reqs[next].arrive <= now) {
            q.submit(next + 1, reqs[next].bytes);
            ++next;
        }
        std::vector<std::pair<uint64_t, uint64_t>> ad;
        q.admit(ad);
        for (auto& a : ad) {
            CHECK(a.first == admitted_order + 1);  // admission strictly in arrival order
            admitted_order = a.first;
            reqs[a.first - 1].admit = now;
            if (running) ++overlapped;
        }
        CHECK(q.arena().in_use() <= q.arena().size());
        for (auto& R : rounds) {
            if (R.busy || q.ready() == 0) continue;
            q.take_round(R.tk);
            uint64_t c = 0;
            for (uint64_t k : R.tk) c += reqs[k - 1].cost;
            R.busy = true;
            R.end = now + c;
            ++running;
        }
        max_running = std::max<uint64_t>(max_running, running);
        CHECK(now < 100000000);
    }
    CHECK(q.arena().in_use() == 0 && q.arena().check());
    CHECK(max_running == (uint64_t)streams);  // rounds overlapped
    CHECK(overlapped > 0);                    // requests joined while others ran
    for (const auto& r : reqs) CHECK(r.done > r.admit && r.admit >= r.arrive);
    printf("policy simulation ok (%llu admitted while running)\n", (unsigned long long)overlapped);
}

int main() {
    arena_basics();
    arena_random();
    admission_fifo();
    admission_rounds_and_cancel();
    policy_simulation();
    printf("OK %d checks\n", g_checks);
    return 0;
}
