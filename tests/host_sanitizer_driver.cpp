// Drives the library's host-only logic, for builds of its host code with
// AddressSanitizer + UndefinedBehaviorSanitizer or ThreadSanitizer
// (tests/test_sanitizers.py): the request server in its fake mode (requests
// submitted from several threads while others poll and wait, passing of a
// blocked large request, the age bound changed while requests run, rejected
// and oversized requests, results handed over once, destruction with
// results left behind), the load balancing of Alg. 3 and the workspace
// footprint.  No GPU is used.  Exits 0 when every check holds.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#include "../include/asci.h"

static int g_bad = 0;
#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            ++g_bad;                                                      \
        }                                                                 \
    } while (0)

static asci_request make_req(int n, int na, int64_t ndets, int64_t k)
{
    asci_request r{};
    r.norb = n;
    r.nalpha = na;
    r.nbeta = na;
    r.ndets = ndets;
    r.k = k;
    r.E0 = -1.0;
    asci_options_default(&r.opt);
    return r;
}

static void balance_checks()
{
    uint64_t x = 12345;
    for (int trial = 0; trial < 50; ++trial) {
        const int64_t m = 1 + (int64_t)(x % 300);
        const int32_t npe = 1 + (int32_t)((x >> 20) % 17);
        std::vector<int64_t> counts((size_t)m);
        int64_t total = 0, mx = 0;
        for (auto &c : counts) {
            x = x * 6364136223846793005ull + 1442695040888963407ull;
            c = (int64_t)((x >> 33) % 100000);
            total += c;
            mx = c > mx ? c : mx;
        }
        std::vector<int32_t> owner((size_t)m, -1);
        std::vector<int64_t> load((size_t)npe, -1);
        CHECK(asci_balance_classes(counts.data(), m, npe, owner.data(), load.data()) == ASCI_OK);
        std::vector<int64_t> sum((size_t)npe, 0);
        for (int64_t i = 0; i < m; ++i) {
            CHECK(owner[(size_t)i] >= 0 && owner[(size_t)i] < npe);
            if (owner[(size_t)i] >= 0 && owner[(size_t)i] < npe) sum[(size_t)owner[(size_t)i]] += counts[(size_t)i];
        }
        int64_t s = 0, lmax = 0;
        for (int32_t q = 0; q < npe; ++q) {
            CHECK(sum[(size_t)q] == load[(size_t)q]);
            s += load[(size_t)q];
            lmax = load[(size_t)q] > lmax ? load[(size_t)q] : lmax;
        }
        CHECK(s == total);
        // greedy list scheduling: at most the mean plus the largest item
        CHECK(lmax * npe <= total + (int64_t)npe * mx);
    }
    CHECK(asci_balance_classes(nullptr, 3, 2, nullptr, nullptr) != ASCI_OK);
}

static void footprint_checks()
{
    int64_t prev = 0;
    for (int64_t nd : {10, 1000, 100000}) {
        asci_request r = make_req(30, 12, nd, 10 * nd);
        const int64_t f = asci_request_footprint(&r);
        CHECK(f > prev);
        prev = f;
    }
    asci_request big = make_req(64, 20, 1000, 10);
    CHECK(asci_request_footprint(&big) > 0);
}

static void server_checks()
{
    asci_server *srv = nullptr;
    CHECK(asci_server_create_fake(4000000000ll, 3, 1e-5, &srv) == ASCI_OK);
    if (!srv) return;
    // invalid and oversized requests are refused at submission
    uint64_t t = 0;
    asci_request bad = make_req(20, 8, 100, 0);
    CHECK(asci_server_submit(srv, &bad, &t) == ASCI_EINVAL);
    asci_request huge = make_req(64, 30, 100000000, 1000000000);
    CHECK(asci_server_submit(srv, &huge, &t) == ASCI_ENOMEM);
    {
        // its failed result waits under its ticket until collected
        asci_result rr{};
        CHECK(asci_server_poll(srv, t, &rr) == ASCI_OK && rr.status == ASCI_ENOMEM);
    }

    // submitters and waiters on several threads, the age bound changed meanwhile
    const int nthr = 4, per = 60;
    std::vector<std::vector<uint64_t>> tickets(nthr);
    std::atomic<int> failures{0};
    std::vector<std::thread> th;
    for (int w = 0; w < nthr; ++w)
        th.emplace_back([&, w] {
            for (int i = 0; i < per; ++i) {
                const int64_t nd = (i % 11 == 0) ? 100000 : (i % 3 == 0 ? 10000 : 1000);
                asci_request r = make_req(20 + 2 * (i % 6), 8 + (i % 3), nd, 10 * nd);
                uint64_t tk = 0;
                if (asci_server_submit(srv, &r, &tk) == ASCI_OK) tickets[(size_t)w].push_back(tk);
                else ++failures;
            }
        });
    std::thread knob([&] {
        for (int i = 0; i < 20; ++i) {
            asci_server_set_param(srv, "age_ms", (i % 2) ? 0.0 : 1e6);
            asci_server_stats st;
            asci_server_get_stats(srv, &st);
            std::this_thread::sleep_for(std::chrono::milliseconds(1));
        }
    });
    for (auto &x : th) x.join();
    knob.join();
    CHECK(failures.load() == 0);
    std::vector<std::thread> waiters;
    std::atomic<int> done{0}, wrong{0};
    for (int w = 0; w < nthr; ++w)
        waiters.emplace_back([&, w] {
            for (size_t i = 0; i < tickets[(size_t)w].size(); ++i) {
                asci_result res{};
                const uint64_t tk = tickets[(size_t)w][i];
                int rc = (i % 2) ? asci_server_wait(srv, tk, &res) : ASCI_EAGAIN;
                while (rc == ASCI_EAGAIN) rc = asci_server_poll(srv, tk, &res);
                if (rc == ASCI_OK && res.status == ASCI_OK) ++done;
                else ++wrong;
                // handed over once: a second collection is refused
                asci_result again{};
                if (asci_server_poll(srv, tk, &again) != ASCI_EINVAL) ++wrong;
            }
        });
    for (auto &x : waiters) x.join();
    CHECK(done.load() == nthr * per);
    CHECK(wrong.load() == 0);
    asci_server_stats st{};
    CHECK(asci_server_get_stats(srv, &st) == ASCI_OK);
    CHECK(st.completed == nthr * per);
    CHECK(st.held_results == 0);
    CHECK(st.max_running >= 1 && st.max_running <= 3);
    CHECK(st.peak_bytes <= 4000000000ll);
    // results left uncollected are released with the server
    for (int i = 0; i < 10; ++i) {
        asci_request r = make_req(20, 8, 1000, 10000);
        asci_server_submit(srv, &r, &t);
    }
    CHECK(asci_server_destroy(srv) == ASCI_OK);
}

int main()
{
    balance_checks();
    footprint_checks();
    server_checks();
    std::printf("host sanitizer driver: %s\n", g_bad ? "FAILED" : "ok");
    return g_bad ? 1 : 0;
}
