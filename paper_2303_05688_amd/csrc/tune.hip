// Per-shape tuning of the search: the LDS bucket capacity of the finish
// ("finish_cap", the sort-and-accumulate tile) chosen by timing, per device
// architecture, orbital count, alpha electron count and pair-count bucket
// (floor(log2 pairs)), kept for the process and optionally saved to and
// loaded from a text file (one "arch norb nalpha bucket finish_cap" line per
// shape).  Searches on a context with "use_tuned" = 1 (default) take the
// tuned capacity of their shape when one is recorded, else the context's.
// The capacity changes speed only, never results.
#include "asci_internal.h"

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <tuple>

namespace asci {

namespace {

using Key = std::tuple<std::string, int, int, int>;

std::mutex g_tune_mu;
std::map<Key, int> g_tune;

std::map<int, std::string> g_arch;  // per device, read once (guarded by g_tune_mu)

std::string arch_of_locked(int device)
{
    auto it = g_arch.find(device);
    if (it != g_arch.end()) return it->second;
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, device) != hipSuccess) {
        (void)hipGetLastError();
        return "unknown";  // not kept: a device may appear later
    }
    std::string a(p.gcnArchName);
    const size_t c = a.find(':');  // drop feature suffixes (":sramecc+:xnack-")
    a = c == std::string::npos ? a : a.substr(0, c);
    g_arch[device] = a;
    return a;
}

int bucket_of(uint64_t pairs) { return pairs ? 63 - __builtin_clzll(pairs) : 0; }

Key key_of_locked(int device, int norb, int na, uint64_t pairs)
{
    return Key{arch_of_locked(device), norb, na, bucket_of(pairs)};
}

}  // namespace

int effective_finish_cap(const asci_ctx *ctx, int norb, int na, uint64_t pairs)
{
    if (!ctx->use_tuned) return ctx->finish_cap;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (g_tune.empty()) return ctx->finish_cap;
    auto it = g_tune.find(key_of_locked(ctx->device, norb, na, pairs));
    return it == g_tune.end() ? ctx->finish_cap : it->second;
}

}  // namespace asci

using namespace asci;

extern "C" {

int asci_tune_shapes(asci_ctx *ctx, const asci_request *reqs, int nreq, int *out_tuned)
{
    try {
        require(ctx != nullptr && (nreq == 0 || reqs != nullptr) && nreq >= 0, ASCI_EINVAL, "bad arguments");
        ASCI_HIP(hipSetDevice(ctx->device));
        int tuned = 0;
        std::map<Key, bool> seen;
        // the context's own settings come back however the timing ends
        struct Restore {
            asci_ctx *c;
            int cap, use;
            ~Restore()
            {
                c->finish_cap = cap;
                c->use_tuned = use;
            }
        } restore{ctx, ctx->finish_cap, ctx->use_tuned};
        const int saved_cap = ctx->finish_cap;
        ctx->use_tuned = 0;
        for (int i = 0; i < nreq; ++i) {
            const asci_request &r = reqs[i];
            check_common(r.norb, r.nalpha, r.nbeta, r.ndets);
            require(r.k >= 1 && r.h && r.eri && r.dets && r.coeffs && r.out_dets && r.out_scores, ASCI_EINVAL,
                    "bad request");
            SearchArgs in{r.h, r.eri, r.norb, r.nalpha, r.nbeta, r.dets, r.coeffs, r.ndets, r.E0, resolve(&r.opt)};
            Key key;
            {
                std::lock_guard<std::mutex> lk(g_tune_mu);
                key = key_of_locked(ctx->device, r.norb, r.nalpha, search_pairs(in));
            }
            if (seen.count(key)) continue;
            seen[key] = true;
            double best = 1e300;
            int best_cap = saved_cap;
            for (int cap : {4096, 2048, 1024}) {
                ctx->finish_cap = cap;
                SearchOut out;
                out.k = r.k;
                out.out_dets = r.out_dets;
                out.out_scores = r.out_scores;
                search_device(ctx, in, out, nullptr);  // untimed: workspaces sized
                double t = 1e300;
                for (int rep = 0; rep < 2; ++rep) {
                    const auto t0 = std::chrono::steady_clock::now();
                    search_device(ctx, in, out, nullptr);
                    t = std::min(t, std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
                }
                if (t < best) {
                    best = t;
                    best_cap = cap;
                }
            }
            {
                std::lock_guard<std::mutex> lk(g_tune_mu);
                g_tune[key] = best_cap;
            }
            ++tuned;
        }
        if (out_tuned) *out_tuned = tuned;
        return ASCI_OK;
    } catch (const Error &e) {
        return report_error(e);
    } catch (const std::bad_alloc &) {
        return report_error(Error{ASCI_ENOMEM, "host memory allocation failed"});
    } catch (const std::exception &e) {
        return report_error(Error{ASCI_EDEVICE, e.what()});
    }
}

int asci_tune_record(const char *arch, int norb, int nalpha, int bucket, int finish_cap)
{
    if (!arch || norb < 1 || norb > 64 || nalpha < 0 || nalpha > norb || bucket < 0 || bucket > 63 ||
        !(finish_cap == 1024 || finish_cap == 2048 || finish_cap == 4096))
        return ASCI_EINVAL;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[Key{std::string(arch), norb, nalpha, bucket}] = finish_cap;
    return ASCI_OK;
}

int asci_tune_lookup(int device, int norb, int nalpha, int64_t pairs, int *finish_cap)
{
    if (!finish_cap || pairs < 0) return ASCI_EINVAL;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key_of_locked(device, norb, nalpha, (uint64_t)pairs));
    *finish_cap = it == g_tune.end() ? 0 : it->second;
    return ASCI_OK;
}

int asci_tune_arch(int device, char *buf, int cap)
{
    if (!buf || cap < 1) return ASCI_EINVAL;
    std::string a;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        a = arch_of_locked(device);
    }
    if ((int)a.size() + 1 > cap) return ASCI_EINVAL;
    std::memcpy(buf, a.c_str(), a.size() + 1);
    return ASCI_OK;
}

int asci_tune_clear(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    return ASCI_OK;
}

int asci_tune_save(const char *path)
{
    if (!path) return ASCI_EINVAL;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    FILE *f = std::fopen(path, "w");
    if (!f) return ASCI_EINVAL;
    for (const auto &kv : g_tune)
        std::fprintf(f, "%s %d %d %d %d\n", std::get<0>(kv.first).c_str(), std::get<1>(kv.first),
                     std::get<2>(kv.first), std::get<3>(kv.first), kv.second);
    const bool ok = std::fclose(f) == 0;
    return ok ? ASCI_OK : ASCI_EINVAL;
}

int asci_tune_load(const char *path, int *out_entries)
{
    if (!path) return ASCI_EINVAL;
    FILE *f = std::fopen(path, "r");
    if (!f) return ASCI_EINVAL;
    char arch[128];
    int norb, na, bucket, cap, n = 0, rc = ASCI_OK;
    for (;;) {
        const int got = std::fscanf(f, "%127s %d %d %d %d", arch, &norb, &na, &bucket, &cap);
        if (got == EOF) break;
        if (got != 5 || asci_tune_record(arch, norb, na, bucket, cap) != ASCI_OK) {
            rc = ASCI_EINVAL;
            break;
        }
        ++n;
    }
    std::fclose(f);
    if (out_entries) *out_entries = n;
    return rc;
}

}  // extern "C"
