// CPU unit test of the server's host core (slot arena, admission, batching).
// Built and run by tests/test_serve_core.py; prints "ok" on success.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <vector>

#include "../../paper_1807_08848_amd/csrc/serve_core.h"

using msrs::serve::Arena;
using msrs::serve::Scheduler;

#define CHECK(x)                                                         \
    do {                                                                 \
        if (!(x)) {                                                      \
            std::fprintf(stderr, "%s:%d: CHECK(%s)\n", __FILE__, __LINE__, #x); \
            std::exit(1);                                                \
        }                                                                \
    } while (0)

struct Block { int64_t off, bytes; };

static void arena_random(uint32_t seed) {
    std::mt19937 g(seed);
    const int64_t cap = 1 << 24;
    Arena a(cap);
    CHECK(a.capacity() == cap && a.used() == 0 && a.largest_free() == cap);
    std::vector<Block> live;
    for (int step = 0; step < 20000; ++step) {
        const bool do_alloc = live.empty() || (g() % 100) < 55;
        if (do_alloc) {
            const int64_t bytes = 1 + (int64_t)(g() % (1u << 18));
            const int64_t off = a.alloc(bytes);
            if (off < 0) {
                CHECK(a.largest_free() < Arena::round(bytes));   // refused only when nothing fits
                continue;
            }
            CHECK(off % Arena::kAlign == 0 && off + bytes <= cap);
            for (auto& b : live)   // disjoint from every live block
                CHECK(off + Arena::round(bytes) <= b.off || b.off + Arena::round(b.bytes) <= off);
            live.push_back({off, bytes});
        } else {
            const size_t i = g() % live.size();
            a.release(live[i].off, live[i].bytes);
            live[i] = live.back();
            live.pop_back();
        }
        CHECK(a.consistent());
        int64_t u = 0;
        for (auto& b : live) u += Arena::round(b.bytes);
        CHECK(u == a.used());
    }
    for (auto& b : live) a.release(b.off, b.bytes);
    CHECK(a.used() == 0 && a.free_blocks() == 1 && a.largest_free() == cap && a.consistent());
}

static void arena_first_fit_and_merge() {
    Arena a(4 * 256);
    const int64_t x = a.alloc(256), y = a.alloc(256), z = a.alloc(256), w = a.alloc(256);
    CHECK(x == 0 && y == 256 && z == 512 && w == 768);
    CHECK(a.alloc(1) == -1);
    a.release(y, 256);
    a.release(z, 200);                 // rounds like the allocation did
    CHECK(a.free_blocks() == 1 && a.largest_free() == 512);
    CHECK(a.alloc(512) == 256);        // merged hole is reused
    a.release(x, 1);
    a.release(w, 256);
    a.release(256, 512);
    CHECK(a.free_blocks() == 1 && a.used() == 0);
}

static void scheduler_fifo_admission() {
    // model 0: small (256 B), model 1: large (768 B); capacity 1024 B
    Arena a(1024);
    Scheduler s(2);
    const int64_t bytes[2] = {256, 768};
    const int models[] = {0, 0, 1, 0, 1, 0};
    for (int i = 0; i < 6; ++i) s.push(i, models[i], bytes[models[i]]);
    std::vector<int64_t> off(6, -1);
    auto fit = [&](const Scheduler::Item& it) {
        const int64_t o = a.alloc(it.bytes);
        if (o < 0) return false;
        off[it.id] = o;
        return true;
    };
    auto adm = s.admit(fit);
    // 256 + 256 fit, the large request (768) does not: strict arrival order stops there
    CHECK(adm.size() == 2 && adm[0].id == 0 && adm[1].id == 1);
    CHECK(s.waiting() == 4 && s.ready() == 2);
    auto b = s.form(8);
    CHECK(b.size() == 2 && b[0].model == 0 && b[0].id == 0 && b[1].id == 1);
    CHECK(s.form(8).empty());
    a.release(off[0], bytes[0]);
    CHECK(s.admit(fit).empty());       // 512 free, head needs 768
    a.release(off[1], bytes[0]);
    adm = s.admit(fit);                // 1024 free: id 2 (768) and id 3 (256)
    CHECK(adm.size() == 2 && adm[0].id == 2 && adm[1].id == 3);
    b = s.form(8);                     // oldest admitted first: model 1
    CHECK(b.size() == 1 && b[0].id == 2);
    b = s.form(8);
    CHECK(b.size() == 1 && b[0].id == 3);
    auto rest = s.drop_all();
    CHECK(rest.size() == 2 && s.waiting() == 0 && s.ready() == 0);
}

static void scheduler_batches_are_homogeneous_and_ordered(uint32_t seed) {
    std::mt19937 g(seed);
    Scheduler s(3);
    std::vector<int> model(500);
    for (int i = 0; i < 500; ++i) {
        model[i] = g() % 3;
        s.push(i, model[i], 1);
    }
    CHECK(s.admit([](const Scheduler::Item&) { return true; }).size() == 500);
    std::set<int64_t> seen;
    int64_t last[3] = {-1, -1, -1};
    for (;;) {
        auto b = s.form(7);
        if (b.empty()) break;
        CHECK(b.size() <= 7);
        for (auto& it : b) {
            CHECK(it.model == b[0].model);      // one model per batch
            CHECK(it.id > last[it.model]);      // arrival order within a model
            last[it.model] = it.id;
            CHECK(seen.insert(it.id).second);   // each request once
        }
    }
    CHECK(seen.size() == 500);
}

int main() {
    arena_first_fit_and_merge();
    for (uint32_t seed = 1; seed <= 4; ++seed) arena_random(seed);
    scheduler_fifo_admission();
    for (uint32_t seed = 1; seed <= 4; ++seed) scheduler_batches_are_homogeneous_and_ordered(seed);
    std::printf("ok\n");
    return 0;
}
