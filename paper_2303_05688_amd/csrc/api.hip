// C ABI of the ASCI search library: argument checks, contexts, host-buffer
// staging, and translation of internal errors into return codes.
#include "asci_internal.h"

#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <stdexcept>

namespace asci {

void Arena::reserve(size_t bytes)
{
    if (bytes <= cap_) return;
    if (fixed_) throw Error{ASCI_ENOMEM, "request larger than the fixed scratch region"};
    const size_t grown = cap_ + cap_ / 4;  // grow by a quarter at least: fewer reallocations
    release();
    auto round = [](size_t b) { return (b + ((size_t)1 << 20) - 1) & ~(((size_t)1 << 20) - 1); };
    void *p = nullptr;
    size_t got = round(std::max(bytes, grown));
    hipError_t e = hipMalloc(&p, got);
    if (e != hipSuccess && got > round(bytes)) {
        (void)hipGetLastError();
        got = round(bytes);
        e = hipMalloc(&p, got);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error{ASCI_ENOMEM, "hipMalloc of the workspace failed"};
    }
    base_ = (char *)p;
    cap_ = got;
    used_ = 0;
}

void Arena::release()
{
    if (base_ && !fixed_) (void)hipFree(base_);
    base_ = nullptr;
    cap_ = used_ = 0;
    fixed_ = false;
}

void HostStage::reserve(size_t b)
{
    if (b <= bytes) return;
    if (fixed) throw Error{ASCI_ENOMEM, "host staging larger than its fixed region"};
    if (ptr) (void)hipHostFree(ptr);
    ptr = nullptr;
    bytes = 0;
    ASCI_HIP(hipHostMalloc(&ptr, b, hipHostMallocDefault));
    bytes = b;
}

HostStage::~HostStage()
{
    if (ptr && !fixed) (void)hipHostFree(ptr);
}

namespace {

thread_local std::string g_last_error;

int fail(const Error &e)
{
    g_last_error = e.what;
    return e.code;
}

}  // namespace

int report_error(const Error &e) { return fail(e); }

void check_common(int norb, int nalpha, int nbeta, int64_t ndets)
{
    require(norb >= 1 && norb <= 64, ASCI_EINVAL, "norb must be in [1, 64]");
    require(nalpha >= 0 && nalpha <= norb && nbeta >= 0 && nbeta <= norb, ASCI_EINVAL,
            "nalpha and nbeta must be in [0, norb]");
    require(ndets >= 1 && ndets < ((int64_t)1 << 31), ASCI_EINVAL, "ndets must be in [1, 2^31)");
}

asci_options resolve(const asci_options *opt)
{
    asci_options o;
    asci_options_default(&o);
    if (opt) o = *opt;
    require(o.constraint_level >= 1 && o.constraint_level <= 6, ASCI_EINVAL, "constraint_level must be in [1, 6]");
    require(o.split_pairs >= 0, ASCI_EINVAL, "split_pairs must be >= 0");
    require(o.ncore >= 0, ASCI_EINVAL, "ncore must be >= 0");
    require(o.pair_buffer_bytes >= 0, ASCI_EINVAL, "pair_buffer_bytes must be >= 0");
    require(!(o.eps < 0.0) && o.eps == o.eps, ASCI_EINVAL, "eps must be >= 0");
    return o;
}

namespace {

struct Staging {
    Arena io;
};

std::mutex g_mu;
std::map<int, std::unique_ptr<asci_ctx>> g_ctx;
std::map<int, std::unique_ptr<Staging>> g_io;

}  // namespace

}  // namespace asci

using namespace asci;

extern "C" {

int asci_version(void) { return (1 << 16) | 0; }

const char *asci_strerror(int code)
{
    switch (code) {
    case ASCI_OK: return "success";
    case ASCI_EINVAL: return "invalid argument";
    case ASCI_ENOMEM: return "out of memory or capacity";
    case ASCI_EDEVICE: return "HIP device error";
    default: return "unknown error";
    }
}

const char *asci_last_error(void) { return g_last_error.c_str(); }

void asci_options_default(asci_options *opt)
{
    if (!opt) return;
    opt->ncore = 0;
    opt->eps = 0.0;
    opt->constraint_level = 3;
    opt->ecore = 0.0;
    opt->pair_buffer_bytes = 0;
    opt->split_pairs = 0;
}

int asci_ctx_create(int device, asci_ctx **out)
{
    try {
        require(out != nullptr, ASCI_EINVAL, "null output pointer");
        int ndev = 0;
        ASCI_HIP(hipGetDeviceCount(&ndev));
        require(device >= 0 && device < ndev, ASCI_EINVAL, "no such device");
        ASCI_HIP(hipSetDevice(device));
        asci_ctx *c = new asci_ctx();
        c->device = device;
        *out = c;
        return ASCI_OK;
    } catch (const Error &e) {
        return fail(e);
    } catch (const std::bad_alloc &) {
        return fail(Error{ASCI_ENOMEM, "host memory allocation failed"});
    } catch (const std::exception &e) {
        return fail(Error{ASCI_EDEVICE, e.what()});
    }
}

int asci_ctx_destroy(asci_ctx *ctx)
{
    if (!ctx) return ASCI_OK;
    try {
        ASCI_HIP(hipSetDevice(ctx->device));
        ASCI_HIP(hipDeviceSynchronize());
    } catch (const Error &e) {
        delete ctx;
        return fail(e);
    }
    delete ctx;
    return ASCI_OK;
}

int asci_ctx_set_param(asci_ctx *ctx, const char *name, int64_t value)
{
    try {
        require(ctx != nullptr && name != nullptr, ASCI_EINVAL, "null argument");
        const std::string key(name);
        if (key == "finish_cap") {
            require(value == 1024 || value == 2048 || value == 4096, ASCI_EINVAL,
                    "finish_cap must be 1024, 2048 or 4096");
            ctx->finish_cap = (int)value;
            return ASCI_OK;
        }
        if (key == "batch_slots") {
            require(value >= 1 && value <= 8, ASCI_EINVAL, "batch_slots must be in [1, 8]");
            ctx->batch_slots = (int)value;
            return ASCI_OK;
        }
        if (key == "spin_tables") {
            require(value == 0 || value == 1, ASCI_EINVAL, "spin_tables must be 0 or 1");
            ctx->spin_tables = (int)value;
            return ASCI_OK;
        }
        if (key == "use_tuned") {
            require(value == 0 || value == 1, ASCI_EINVAL, "use_tuned must be 0 or 1");
            ctx->use_tuned = (int)value;
            return ASCI_OK;
        }
        if (key == "batch_solo_pairs") {
            require(value >= 0, ASCI_EINVAL, "batch_solo_pairs must be >= 0");
            ctx->batch_solo_pairs = value;
            return ASCI_OK;
        }
        if (key == "batch_graph") {
            require(value == 0 || value == 1, ASCI_EINVAL, "batch_graph must be 0 or 1");
            ctx->batch_graph = (int)value;
            return ASCI_OK;
        }
        if (key == "fault_test") {
            require(value == 0 || value == 1, ASCI_EINVAL, "fault_test must be 0 or 1");
            ctx->fault_test = (int)value;
            return ASCI_OK;
        }
        if (key == "release_workspace") {
            require(value == 1, ASCI_EINVAL, "release_workspace takes the value 1");
            ASCI_HIP(hipSetDevice(ctx->device));
            ASCI_HIP(hipDeviceSynchronize());
            if (ctx->batch_pool) ctx->batch_pool_free(ctx->batch_pool);
            ctx->batch_pool = nullptr;
            ctx->batch_pool_slots = ctx->batch_pool_cap = 0;
            if (ctx->graph_batch) ctx->graph_batch_free(ctx->graph_batch);
            ctx->graph_batch = nullptr;
            ctx->setup.release();
            ctx->main.release();
            ctx->tables.release();
            return ASCI_OK;
        }
        throw Error{ASCI_EINVAL, "unknown parameter: " + key};
    } catch (const Error &e) {
        return fail(e);
    } catch (const std::bad_alloc &) {
        return fail(Error{ASCI_ENOMEM, "host memory allocation failed"});
    } catch (const std::exception &e) {
        return fail(Error{ASCI_EDEVICE, e.what()});
    }
}

int asci_ctx_get_param(asci_ctx *ctx, const char *name, int64_t *value)
{
    try {
        require(ctx != nullptr && name != nullptr && value != nullptr, ASCI_EINVAL, "null argument");
        const std::string key(name);
        if (key == "finish_cap") *value = ctx->finish_cap;
        else if (key == "batch_slots") *value = ctx->batch_slots;
        else if (key == "spin_tables") *value = ctx->spin_tables;
        else if (key == "fault_test") *value = ctx->fault_test;
        else if (key == "batch_graph") *value = ctx->batch_graph;
        else if (key == "batch_solo_pairs") *value = ctx->batch_solo_pairs;
        else if (key == "use_tuned") *value = ctx->use_tuned;
        else if (key == "last_batches") *value = ctx->last_batches;
        else if (key == "last_finals") *value = ctx->last_finals;
        else if (key == "last_levels") *value = ctx->last_levels;
        else if (key == "last_candidates") *value = ctx->last_candidates;
        else throw Error{ASCI_EINVAL, "unknown parameter: " + key};
        return ASCI_OK;
    } catch (const Error &e) {
        return fail(e);
    } catch (const std::bad_alloc &) {
        return fail(Error{ASCI_ENOMEM, "host memory allocation failed"});
    } catch (const std::exception &e) {
        return fail(Error{ASCI_EDEVICE, e.what()});
    }
}

int asci_ctx_set_profiling(asci_ctx *ctx, int enable)
{
    try {
        require(ctx != nullptr, ASCI_EINVAL, "null context");
        ASCI_HIP(hipSetDevice(ctx->device));
        ctx->prof.reset();
        ctx->prof.on = enable != 0;
        return ASCI_OK;
    } catch (const Error &e) {
        return fail(e);
    } catch (const std::bad_alloc &) {
        return fail(Error{ASCI_ENOMEM, "host memory allocation failed"});
    } catch (const std::exception &e) {
        return fail(Error{ASCI_EDEVICE, e.what()});
    }
}

int asci_ctx_profile_only(asci_ctx *ctx, const char *kernel)
{
    try {
        require(ctx != nullptr, ASCI_EINVAL, "null context");
        ctx->prof.only = kernel ? std::string(kernel) : std::string();
        return ASCI_OK;
    } catch (const Error &e) {
        return fail(e);
    } catch (const std::bad_alloc &) {
        return fail(Error{ASCI_ENOMEM, "host memory allocation failed"});
    } catch (const std::exception &e) {
        return fail(Error{ASCI_EDEVICE, e.what()});
    }
}

int asci_ctx_profile_entry(asci_ctx *ctx, int index, char *name, int name_cap, double *total_ms,
                           int64_t *launches, double *bytes)
{
    try {
        require(ctx != nullptr, ASCI_EINVAL, "null context");
        ctx->prof.collect();
        require(index >= 0 && index < (int)ctx->prof.entries.size(), ASCI_EINVAL, "no such profile entry");
        const ProfEntry &e = ctx->prof.entries[(size_t)index];
        if (name && name_cap > 0) {
            std::strncpy(name, e.name.c_str(), (size_t)name_cap - 1);
            name[name_cap - 1] = 0;
        }
        if (total_ms) *total_ms = e.ms;
        if (launches) *launches = e.launches;
        if (bytes) *bytes = e.bytes;
        return ASCI_OK;
    } catch (const Error &e) {
        return fail(e);
    } catch (const std::bad_alloc &) {
        return fail(Error{ASCI_ENOMEM, "host memory allocation failed"});
    } catch (const std::exception &e) {
        return fail(Error{ASCI_EDEVICE, e.what()});
    }
}

int asci_search_device(asci_ctx *ctx, const double *d_h, const double *d_eri, int norb, int nalpha, int nbeta,
                       const uint64_t *d_dets, const double *d_coeffs, int64_t ndets, double E0, int64_t k,
                       const asci_options *opt, uint64_t *d_out_dets, double *d_out_scores, int64_t *out_count,
                       void *stream)
{
    try {
        require(ctx && d_h && d_eri && d_dets && d_coeffs && d_out_dets && d_out_scores && out_count, ASCI_EINVAL,
                "null pointer argument");
        check_common(norb, nalpha, nbeta, ndets);
        require(k >= 1, ASCI_EINVAL, "k must be >= 1");
        ASCI_HIP(hipSetDevice(ctx->device));
        SearchArgs in{d_h, d_eri, norb, nalpha, nbeta, d_dets, d_coeffs, ndets, E0, resolve(opt)};
        SearchOut out;
        out.k = k;
        out.out_dets = d_out_dets;
        out.out_scores = d_out_scores;
        search_device(ctx, in, out, (hipStream_t)stream);
        *out_count = out.count;
        return ASCI_OK;
    } catch (const Error &e) {
        return fail(e);
    } catch (const std::bad_alloc &) {
        return fail(Error{ASCI_ENOMEM, "host memory allocation failed"});
    } catch (const std::exception &e) {
        return fail(Error{ASCI_EDEVICE, e.what()});
    }
}

int asci_search_async(asci_ctx *ctx, const asci_request *req, asci_async_result *d_result, void *stream)
{
    try {
        require(ctx != nullptr && req != nullptr && d_result != nullptr, ASCI_EINVAL, "null argument");
        check_common(req->norb, req->nalpha, req->nbeta, req->ndets);
        require(req->h && req->eri && req->dets && req->coeffs && req->out_dets && req->out_scores, ASCI_EINVAL,
                "null buffer in the request");
        ASCI_HIP(hipSetDevice(ctx->device));
        SearchArgs in{req->h, req->eri, req->norb, req->nalpha, req->nbeta, req->dets, req->coeffs, req->ndets,
                      req->E0, resolve(&req->opt)};
        search_async(ctx, in, req->k, req->out_dets, req->out_scores, d_result, (hipStream_t)stream);
        return ASCI_OK;
    } catch (const Error &e) {
        return fail(e);
    } catch (const std::bad_alloc &) {
        return fail(Error{ASCI_ENOMEM, "host memory allocation failed"});
    } catch (const std::exception &e) {
        return fail(Error{ASCI_EDEVICE, e.what()});
    }
}

int asci_request_async_bytes(asci_ctx *ctx, const asci_request *req, int64_t *out_bytes)
{
    try {
        require(ctx != nullptr && req != nullptr && out_bytes != nullptr, ASCI_EINVAL, "null argument");
        check_common(req->norb, req->nalpha, req->nbeta, req->ndets);
        SearchArgs in{req->h, req->eri, req->norb, req->nalpha, req->nbeta, req->dets, req->coeffs, req->ndets,
                      req->E0, resolve(&req->opt)};
        *out_bytes = (int64_t)search_async_bytes(in, req->k, ctx->finish_cap, ctx->spin_tables != 0);
        return ASCI_OK;
    } catch (const Error &e) {
        return fail(e);
    } catch (const std::exception &e) {
        return fail(Error{ASCI_EDEVICE, e.what()});
    }
}

int asci_candidates_device(asci_ctx *ctx, const double *d_h, const double *d_eri, int norb, int nalpha,
                           int nbeta, const uint64_t *d_dets, const double *d_coeffs, int64_t ndets, double E0,
                           const asci_options *opt, int64_t capacity, uint64_t *d_out_dets, double *d_out_num,
                           double *d_out_scores, int64_t *out_count, void *stream)
{
    try {
        require(ctx && d_h && d_eri && d_dets && d_coeffs && out_count, ASCI_EINVAL, "null pointer argument");
        require(capacity == 0 || (d_out_dets && d_out_num && d_out_scores), ASCI_EINVAL, "null output buffer");
        require(capacity >= 0, ASCI_EINVAL, "capacity must be >= 0");
        check_common(norb, nalpha, nbeta, ndets);
        ASCI_HIP(hipSetDevice(ctx->device));
        SearchArgs in{d_h, d_eri, norb, nalpha, nbeta, d_dets, d_coeffs, ndets, E0, resolve(opt)};
        SearchOut out;
        out.k = 0;
        out.capacity = capacity;
        out.out_dets = d_out_dets;
        out.out_num = d_out_num;
        out.out_scores = d_out_scores;
        search_device(ctx, in, out, (hipStream_t)stream);
        *out_count = out.count;
        if (out.count > capacity) throw Error{ASCI_ENOMEM, "output capacity below the candidate count"};
        return ASCI_OK;
    } catch (const Error &e) {
        return fail(e);
    } catch (const std::bad_alloc &) {
        return fail(Error{ASCI_ENOMEM, "host memory allocation failed"});
    } catch (const std::exception &e) {
        return fail(Error{ASCI_EDEVICE, e.what()});
    }
}

int asci_pt2_device(asci_ctx *ctx, const double *d_h, const double *d_eri, int norb, int nalpha, int nbeta,
                    const uint64_t *d_dets, const double *d_coeffs, int64_t ndets, double E0,
                    const asci_options *opt, double *out_energy, int64_t *out_count, void *stream)
{
    try {
        require(ctx && d_h && d_eri && d_dets && d_coeffs && out_energy && out_count, ASCI_EINVAL,
                "null pointer argument");
        check_common(norb, nalpha, nbeta, ndets);
        ASCI_HIP(hipSetDevice(ctx->device));
        SearchArgs in{d_h, d_eri, norb, nalpha, nbeta, d_dets, d_coeffs, ndets, E0, resolve(opt)};
        SearchOut out;
        out.k = 0;
        out.pt2 = true;
        search_device(ctx, in, out, (hipStream_t)stream);
        *out_energy = out.pt2_energy;
        *out_count = out.count;
        return ASCI_OK;
    } catch (const Error &e) {
        return fail(e);
    } catch (const std::bad_alloc &) {
        return fail(Error{ASCI_ENOMEM, "host memory allocation failed"});
    } catch (const std::exception &e) {
        return fail(Error{ASCI_EDEVICE, e.what()});
    }
}

// ---------------------------------------------------------------- variational step and loop
struct asci_hmat {
    asci::HMat H;
};

int asci_hmat_build_device(asci_ctx *ctx, const double *d_h, const double *d_eri, int norb, int nalpha,
                           int nbeta, const uint64_t *d_dets, int64_t ndets, double ecore, asci_hmat **out,
                           void *stream)
{
    try {
        require(ctx && d_h && d_eri && d_dets && out, ASCI_EINVAL, "null pointer argument");
        check_common(norb, nalpha, nbeta, ndets);
        ASCI_HIP(hipSetDevice(ctx->device));
        std::unique_ptr<asci_hmat> m(new asci_hmat);
        hmat_build(ctx, d_h, d_eri, norb, nalpha, nbeta, d_dets, ndets, ecore, m->H, (hipStream_t)stream);
        *out = m.release();
        return ASCI_OK;
    } catch (const Error &e) {
        return fail(e);
    } catch (const std::bad_alloc &) {
        return fail(Error{ASCI_ENOMEM, "host memory allocation failed"});
    } catch (const std::exception &e) {
        return fail(Error{ASCI_EDEVICE, e.what()});
    }
}

int asci_hmat_info(const asci_hmat *H, int64_t *nrows, int64_t *nnz)
{
    try {
        require(H && nrows && nnz, ASCI_EINVAL, "null pointer argument");
        *nrows = H->H.nrows;
        *nnz = H->H.nnz;
        return ASCI_OK;
    } catch (const Error &e) {
        return fail(e);
    } catch (const std::bad_alloc &) {
        return fail(Error{ASCI_ENOMEM, "host memory allocation failed"});
    } catch (const std::exception &e) {
        return fail(Error{ASCI_EDEVICE, e.what()});
    }
}

int asci_hmat_export(const asci_hmat *H, int64_t *d_rowptr, int32_t *d_cols, double *d_vals, void *stream)
{
    try {
        require(H && d_rowptr && d_cols && d_vals, ASCI_EINVAL, "null pointer argument");
        ASCI_HIP(hipSetDevice(H->H.device));
        const hipStream_t s = (hipStream_t)stream;
        ASCI_HIP(hipMemcpyAsync(d_rowptr, H->H.rowptr, (size_t)(H->H.nrows + 1) * sizeof(int64_t),
                                hipMemcpyDeviceToDevice, s));
        if (H->H.nnz) {
            ASCI_HIP(hipMemcpyAsync(d_cols, H->H.cols, (size_t)H->H.nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
            ASCI_HIP(hipMemcpyAsync(d_vals, H->H.vals, (size_t)H->H.nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
        }
        ASCI_HIP(hipStreamSynchronize(s));
        return ASCI_OK;
    } catch (const Error &e) {
        return fail(e);
    } catch (const std::bad_alloc &) {
        return fail(Error{ASCI_ENOMEM, "host memory allocation failed"});
    } catch (const std::exception &e) {
        return fail(Error{ASCI_EDEVICE, e.what()});
    }
}

int asci_hmat_matvec_device(const asci_hmat *H, const double *d_x, double *d_y, void *stream)
{
    try {
        require(H && d_x && d_y, ASCI_EINVAL, "null pointer argument");
        ASCI_HIP(hipSetDevice(H->H.device));
        hmat_matvec(H->H, d_x, d_y, (hipStream_t)stream);
        return ASCI_OK;
    } catch (const Error &e) {
        return fail(e);
    } catch (const std::bad_alloc &) {
        return fail(Error{ASCI_ENOMEM, "host memory allocation failed"});
    } catch (const std::exception &e) {
        return fail(Error{ASCI_EDEVICE, e.what()});
    }
}

void asci_hmat_destroy(asci_hmat *H) { delete H; }

int asci_davidson_device(asci_ctx *ctx, const asci_hmat *H, const double *d_guess, int32_t max_subspace,
                         int32_t max_iter, double tol, double *out_energy, double *d_vec, double *out_resid,
                         int32_t *out_iters, void *stream)
{
    try {
        require(ctx && H && out_energy && d_vec && out_resid && out_iters, ASCI_EINVAL, "null pointer argument");
        require(max_subspace >= 2 && max_subspace <= 48, ASCI_EINVAL, "max_subspace must be in [2, 48]");
        require(max_iter >= 1 && tol >= 0.0, ASCI_EINVAL, "max_iter must be >= 1 and tol >= 0");
        require(H->H.device == ctx->device, ASCI_EINVAL, "matrix and context on different devices");
        ASCI_HIP(hipSetDevice(ctx->device));
        DavidsonOpts o;
        o.max_subspace = max_subspace;
        o.max_iter = max_iter;
        o.tol = tol;
        const DavidsonOut r = davidson(ctx, H->H, d_guess, o, d_vec, (hipStream_t)stream);
        *out_energy = r.energy;
        *out_resid = r.resid;
        *out_iters = r.iters;
        return ASCI_OK;
    } catch (const Error &e) {
        return fail(e);
    } catch (const std::bad_alloc &) {
        return fail(Error{ASCI_ENOMEM, "host memory allocation failed"});
    } catch (const std::exception &e) {
        return fail(Error{ASCI_EDEVICE, e.what()});
    }
}

void asci_loop_options_default(asci_loop_options *opt)
{
    if (!opt) return;
    opt->ncore = 0;
    opt->ntdets = 1000;
    opt->max_iter = 10;
    opt->e_tol = 1e-6;
    opt->davidson_subspace = 24;
    opt->davidson_max_iter = 200;
    opt->davidson_tol = 1e-8;
    opt->pt2 = 0;
    asci_options_default(&opt->search);
}

static LoopArgs loop_args(const double *d_h, const double *d_eri, int norb, int nalpha, int nbeta,
                          const asci_loop_options *opt)
{
    LoopArgs a;
    a.h = d_h;
    a.eri = d_eri;
    a.n = norb;
    a.na = nalpha;
    a.nb = nbeta;
    asci_loop_options_default(&a.opt);
    if (opt) a.opt = *opt;
    a.opt.search = resolve(&a.opt.search);
    require(a.opt.ntdets >= 1 && a.opt.ntdets < ((int64_t)1 << 31), ASCI_EINVAL, "ntdets must be in [1, 2^31)");
    require(a.opt.ncore >= 0 && a.opt.max_iter >= 1 && a.opt.e_tol >= 0.0, ASCI_EINVAL,
            "ncore >= 0, max_iter >= 1 and e_tol >= 0 required");
    require(a.opt.davidson_subspace >= 2 && a.opt.davidson_subspace <= 48 && a.opt.davidson_max_iter >= 1 &&
                a.opt.davidson_tol >= 0.0,
            ASCI_EINVAL, "Davidson options out of range");
    a.dav.max_subspace = a.opt.davidson_subspace;
    a.dav.max_iter = a.opt.davidson_max_iter;
    a.dav.tol = a.opt.davidson_tol;
    return a;
}

int asci_loop_step_device(asci_ctx *ctx, const double *d_h, const double *d_eri, int norb, int nalpha, int nbeta,
                          const uint64_t *d_dets, const double *d_coeffs, int64_t ndets, double Ek,
                          const asci_loop_options *opt, uint64_t *d_out_dets, double *d_out_coeffs,
                          int64_t *out_ndets, asci_loop_iter *info, void *stream)
{
    try {
        require(ctx && d_h && d_eri && d_dets && d_coeffs && d_out_dets && d_out_coeffs && out_ndets && info,
                ASCI_EINVAL, "null pointer argument");
        check_common(norb, nalpha, nbeta, ndets);
        ASCI_HIP(hipSetDevice(ctx->device));
        const LoopArgs a = loop_args(d_h, d_eri, norb, nalpha, nbeta, opt);
        LoopIter it{};
        int64_t nn = 0;
        loop_step(ctx, a, d_dets, d_coeffs, ndets, Ek, d_out_dets, d_out_coeffs, nn, it, (hipStream_t)stream);
        *out_ndets = nn;
        *info = it;
        return ASCI_OK;
    } catch (const Error &e) {
        return fail(e);
    } catch (const std::bad_alloc &) {
        return fail(Error{ASCI_ENOMEM, "host memory allocation failed"});
    } catch (const std::exception &e) {
        return fail(Error{ASCI_EDEVICE, e.what()});
    }
}

int asci_run_device(asci_ctx *ctx, const double *d_h, const double *d_eri, int norb, int nalpha, int nbeta,
                    const uint64_t *d_dets0, const double *d_coeffs0, int64_t ndets0, const asci_loop_options *opt,
                    uint64_t *d_out_dets, double *d_out_coeffs, int64_t *out_ndets, double *out_energy,
                    double *out_pt2, asci_loop_iter *iters, int32_t *out_iters, void *stream)
{
    try {
        require(ctx && d_h && d_eri && d_dets0 && d_coeffs0 && d_out_dets && d_out_coeffs && out_ndets &&
                    out_energy && out_pt2 && iters && out_iters,
                ASCI_EINVAL, "null pointer argument");
        check_common(norb, nalpha, nbeta, ndets0);
        ASCI_HIP(hipSetDevice(ctx->device));
        const LoopArgs a = loop_args(d_h, d_eri, norb, nalpha, nbeta, opt);
        validate_dets(ctx, d_dets0, ndets0, norb, nalpha, nbeta, (hipStream_t)stream);
        std::vector<LoopIter> rec;
        int64_t nn = 0;
        double e = 0.0, p = 0.0;
        loop_run(ctx, a, d_dets0, d_coeffs0, ndets0, d_out_dets, d_out_coeffs, nn, e, p, rec, (hipStream_t)stream);
        *out_ndets = nn;
        *out_energy = e;
        *out_pt2 = p;
        *out_iters = (int32_t)rec.size();
        for (size_t i = 0; i < rec.size(); ++i) iters[i] = rec[i];
        return ASCI_OK;
    } catch (const Error &e) {
        return fail(e);
    } catch (const std::bad_alloc &) {
        return fail(Error{ASCI_ENOMEM, "host memory allocation failed"});
    } catch (const std::exception &e) {
        return fail(Error{ASCI_EDEVICE, e.what()});
    }
}

int asci_class_counts_device(asci_ctx *ctx, int norb, int nalpha, int nbeta, const uint64_t *d_dets,
                             const double *d_coeffs, int64_t ndets, const asci_options *opt, int64_t capacity,
                             uint64_t *h_masks, int64_t *h_counts, int64_t *out_nclasses, void *stream)
{
    try {
        require(ctx && d_dets && d_coeffs && out_nclasses, ASCI_EINVAL, "null pointer argument");
        require(capacity >= 0 && (capacity == 0 || (h_masks && h_counts)), ASCI_EINVAL, "bad output buffers");
        check_common(norb, nalpha, nbeta, ndets);
        const asci_options o = resolve(opt);
        ASCI_HIP(hipSetDevice(ctx->device));
        std::vector<uint64_t> masks, counts;
        class_counts_device(ctx, norb, nalpha, nbeta, d_dets, d_coeffs, ndets, o, masks, counts,
                            (hipStream_t)stream);
        *out_nclasses = (int64_t)masks.size();
        require((int64_t)masks.size() <= capacity, ASCI_ENOMEM, "output capacity below the class count");
        for (size_t i = 0; i < masks.size(); ++i) {
            h_masks[i] = masks[i];
            h_counts[i] = (int64_t)counts[i];
        }
        return ASCI_OK;
    } catch (const Error &e) {
        return fail(e);
    } catch (const std::bad_alloc &) {
        return fail(Error{ASCI_ENOMEM, "host memory allocation failed"});
    } catch (const std::exception &e) {
        return fail(Error{ASCI_EDEVICE, e.what()});
    }
}

int asci_balance_classes(const int64_t *counts, int64_t nclasses, int32_t npe, int32_t *owner, int64_t *load)
{
    try {
        require(counts && owner && load, ASCI_EINVAL, "null pointer argument");
        require(nclasses >= 0 && npe >= 1, ASCI_EINVAL, "nclasses must be >= 0 and npe >= 1");
        for (int64_t c = 0; c < nclasses; ++c) require(counts[c] >= 0, ASCI_EINVAL, "negative class count");
        // a binary heap of (load, element) keeps the arg-min at O(log npe)
        std::vector<std::pair<int64_t, int32_t>> heap((size_t)npe);
        for (int32_t p = 0; p < npe; ++p) heap[(size_t)p] = {0, p};
        auto later = [](const std::pair<int64_t, int32_t> &x, const std::pair<int64_t, int32_t> &y) {
            return x > y;  // min-heap on (load, element)
        };
        for (int32_t p = 0; p < npe; ++p) load[p] = 0;
        for (int64_t c = 0; c < nclasses; ++c) {
            if (counts[c] == 0) {
                owner[c] = -1;
                continue;
            }
            std::pop_heap(heap.begin(), heap.end(), later);
            auto &q = heap.back();
            owner[c] = q.second;
            q.first += counts[c];
            load[q.second] = q.first;
            std::push_heap(heap.begin(), heap.end(), later);
        }
        return ASCI_OK;
    } catch (const Error &e) {
        return fail(e);
    } catch (const std::bad_alloc &) {
        return fail(Error{ASCI_ENOMEM, "host memory allocation failed"});
    } catch (const std::exception &e) {
        return fail(Error{ASCI_EDEVICE, e.what()});
    }
}

int asci_energy_device(asci_ctx *ctx, const double *d_h, const double *d_eri, int norb, int nalpha, int nbeta,
                       const uint64_t *d_dets, const double *d_coeffs, int64_t ndets, double ecore,
                       double *out_energy, void *stream)
{
    try {
        require(ctx && d_h && d_eri && d_dets && d_coeffs && out_energy, ASCI_EINVAL, "null pointer argument");
        check_common(norb, nalpha, nbeta, ndets);
        ASCI_HIP(hipSetDevice(ctx->device));
        validate_dets(ctx, d_dets, ndets, norb, nalpha, nbeta, (hipStream_t)stream);
        *out_energy = energy_device(ctx, d_h, d_eri, norb, d_dets, d_coeffs, ndets, ecore, (hipStream_t)stream);
        return ASCI_OK;
    } catch (const Error &e) {
        return fail(e);
    } catch (const std::bad_alloc &) {
        return fail(Error{ASCI_ENOMEM, "host memory allocation failed"});
    } catch (const std::exception &e) {
        return fail(Error{ASCI_EDEVICE, e.what()});
    }
}

int asci_search(const double *h, const double *eri, int norb, int nalpha, int nbeta, const uint64_t *dets,
                const double *coeffs, int64_t ndets, double E0, int64_t k, const asci_options *opt,
                uint64_t *out_dets, double *out_scores, int64_t *out_count)
{
    try {
        require(h && eri && dets && coeffs && out_dets && out_scores && out_count, ASCI_EINVAL,
                "null pointer argument");
        check_common(norb, nalpha, nbeta, ndets);
        require(k >= 1, ASCI_EINVAL, "k must be >= 1");
        const asci_options o = resolve(opt);
        int dev = 0;
        ASCI_HIP(hipGetDevice(&dev));
        std::lock_guard<std::mutex> lock(g_mu);
        auto &slot = g_ctx[dev];
        if (!slot) {
            asci_ctx *c = nullptr;
            int rc = asci_ctx_create(dev, &c);
            if (rc != ASCI_OK) return rc;
            slot.reset(c);
        }
        auto &io = g_io[dev];
        if (!io) io.reset(new Staging());
        const size_t n = (size_t)norb, nd = (size_t)ndets;
        io->io.reset();
        io->io.reserve(n * n * 8 + n * n * n * n * 8 + nd * 24 + (size_t)k * 24 + 8 * 256);
        io->io.reset();
        double *dh = io->io.take<double>(n * n);
        double *de = io->io.take<double>(n * n * n * n);
        uint64_t *dd = io->io.take<uint64_t>(2 * nd);
        double *dc = io->io.take<double>(nd);
        uint64_t *od = io->io.take<uint64_t>(2 * (size_t)k);
        double *os = io->io.take<double>((size_t)k);
        hipStream_t s = nullptr;
        ASCI_HIP(hipMemcpy(dh, h, n * n * 8, hipMemcpyHostToDevice));
        ASCI_HIP(hipMemcpy(de, eri, n * n * n * n * 8, hipMemcpyHostToDevice));
        ASCI_HIP(hipMemcpy(dd, dets, nd * 16, hipMemcpyHostToDevice));
        ASCI_HIP(hipMemcpy(dc, coeffs, nd * 8, hipMemcpyHostToDevice));
        SearchArgs in{dh, de, norb, nalpha, nbeta, dd, dc, ndets, E0, o};
        SearchOut out;
        out.k = k;
        out.out_dets = od;
        out.out_scores = os;
        search_device(slot.get(), in, out, s);
        if (out.count > 0) {
            ASCI_HIP(hipMemcpy(out_dets, od, (size_t)out.count * 16, hipMemcpyDeviceToHost));
            ASCI_HIP(hipMemcpy(out_scores, os, (size_t)out.count * 8, hipMemcpyDeviceToHost));
        }
        *out_count = out.count;
        return ASCI_OK;
    } catch (const Error &e) {
        return fail(e);
    } catch (const std::bad_alloc &) {
        return fail(Error{ASCI_ENOMEM, "host memory allocation failed"});
    } catch (const std::exception &e) {
        return fail(Error{ASCI_EDEVICE, e.what()});
    }
}

}  // extern "C"
