// The search for callers that cannot allocate device memory (code under HIP
// graph capture, tight serving loops, harnesses that forbid hipMalloc): the
// same pipeline as asci_search_device, with every device buffer carved from a
// fixed scratch region that the library holds from load time, and host
// readbacks staged in a fixed host buffer.
//
// The region is a file-scope device array.  Its name is only a host-side
// stand-in for the device object, so the host never passes it to a kernel or
// a copy: on the first call on a device (with that device current) its
// address there is taken once with hipGetSymbolAddress and kept per device,
// and every carve starts from that address.
#include "asci_internal.h"

#include <cstring>
#include <mutex>
#include <new>
#include <stdexcept>

namespace asci {

namespace {

constexpr size_t kScratchBytes = (size_t)256 << 20;  // 256 MiB per device
constexpr size_t kHostStageBytes = (size_t)1 << 20;  // readbacks of one call
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct NoAllocDevice {
    std::mutex mu;           // one call at a time per device through this entry point
    char *ptr = nullptr;     // the scratch region's address on this device
    asci_ctx *ctx = nullptr; // arenas attached to it, no spin tables, no profiling
    unsigned char *host = nullptr;
};

NoAllocDevice g_dev[kMaxDevices];

// set-up on the device's first call (that device current, d.mu held): the
// region's address
void setup_locked(NoAllocDevice &d, int dev)
{
    if (!d.ptr) {
        void *p = nullptr;
        ASCI_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        require(p != nullptr, ASCI_EDEVICE, "scratch region has no device address");
        // host-side state, created once per device and kept for the process
        d.ctx = new asci_ctx();
        d.ctx->device = dev;
        d.ctx->spin_tables = 0;  // the tables live in an arena of their own; direct evaluation gives the same bits
        d.host = new unsigned char[kHostStageBytes];
        d.ctx->stage.attach(d.host, kHostStageBytes);
        d.ptr = (char *)p;
    }
}

}  // namespace

}  // namespace asci

using namespace asci;

extern "C" int asci_search_device_noalloc(const double *d_h, const double *d_eri, int norb, int nalpha, int nbeta,
                                          const uint64_t *d_dets, const double *d_coeffs, int64_t ndets, double E0,
                                          int64_t k, const asci_options *opt, uint64_t *d_out_dets,
                                          double *d_out_scores, int64_t *out_count, void *stream)
{
    try {
        check_common(norb, nalpha, nbeta, ndets);
        require(k >= 1, ASCI_EINVAL, "k must be >= 1");
        require(d_h && d_eri && d_dets && d_coeffs && d_out_dets && d_out_scores && out_count, ASCI_EINVAL,
                "null argument");
        asci_options o = resolve(opt);
        int dev = 0;
        ASCI_HIP(hipGetDevice(&dev));
        require(dev >= 0 && dev < kMaxDevices, ASCI_EINVAL, "device index out of range");
        NoAllocDevice &d = g_dev[dev];
        std::lock_guard<std::mutex> lk(d.mu);
        setup_locked(d, dev);
        // one class batch holds every pair: the pair buffer is sized from the
        // closed-form count, so no free-memory query or extra batch is needed
        SearchArgs in{d_h, d_eri, norb, nalpha, nbeta, d_dets, d_coeffs, ndets, E0, o};
        const int W = norb <= 32 ? 1 : 2;
        const uint64_t pairs = std::max<uint64_t>(search_pairs(in), 1);
        in.opt.pair_buffer_bytes = (int64_t)(pairs * 2 * (8 * W + 8));
        size_t setup_part = 0;
        const size_t need = search_scratch_bound(in, k, d.ctx->finish_cap, setup_part);
        if (need > kScratchBytes)
            throw Error{ASCI_ENOMEM, "search needs up to " + std::to_string(need) + " bytes of scratch; the "
                                     "allocation-free entry point holds " + std::to_string(kScratchBytes)};
        d.ctx->setup.attach(d.ptr, setup_part);
        d.ctx->main.attach(d.ptr + setup_part, kScratchBytes - setup_part);
        SearchOut out;
        out.k = k;
        out.out_dets = d_out_dets;
        out.out_scores = d_out_scores;
        search_device(d.ctx, in, out, (hipStream_t)stream);
        *out_count = out.count;
        return ASCI_OK;
    } catch (const Error &e) {
        return report_error(e);
    } catch (const std::bad_alloc &) {
        return report_error(Error{ASCI_ENOMEM, "host memory allocation failed"});
    } catch (const std::exception &e) {
        return report_error(Error{ASCI_EDEVICE, e.what()});
    }
}
