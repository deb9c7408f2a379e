// C-ABI entry points of the dctplus library.  Argument checks happen on the
// host before any device work; every HIP error becomes DCTPLUS_EDEVICE.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <new>
#include <string>

#include "common.h"

// Scratch of dctplus_grad_noalloc: one fixed device array per GPU, held until
// the process ends.  Host code never uses its name as an address: the device
// address of each GPU's copy is looked up once per device (scratch_ptr).
constexpr size_t kStaticScratchBytes = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace dctplus {

static thread_local char g_err[512] = "";

dctplus_status fail(dctplus_status s, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

dctplus_status hip_fail(hipError_t e, const char *what) {
    return fail(DCTPLUS_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

dctplus_status stream_work(dctplus_plan_s *p, hipStream_t s, size_t bytes, void **out) {
    std::lock_guard<std::mutex> lock(p->work_mu);
    dctplus_plan_s::StreamWork *w = nullptr;
    for (auto &e : p->works)
        if (e.stream == s) w = &e;
    if (!w) {
        p->works.push_back({s, nullptr, 0});
        w = &p->works.back();
    }
    if (w->bytes < bytes) {
        if (w->ptr) {
            // this stream's earlier calls must be done with the old buffer before it goes
            hipError_t e = hipStreamSynchronize(s);
            if (e != hipSuccess) return hip_fail(e, "synchronize before workspace growth");
            (void)hipFree(w->ptr);
            w->ptr = nullptr;
            w->bytes = 0;
        }
        hipError_t e = hipMalloc(&w->ptr, bytes);
        if (e != hipSuccess) {
            w->ptr = nullptr;
            (void)hipGetLastError();
            return fail(DCTPLUS_ENOMEM, "hipMalloc(%zu) for the workspace failed", bytes);
        }
        w->bytes = bytes;
    }
    *out = w->ptr;
    return DCTPLUS_OK;
}

void release_works(dctplus_plan_s *p) {
    std::lock_guard<std::mutex> lock(p->work_mu);
    for (auto &e : p->works)
        if (e.ptr) (void)hipFree(e.ptr);
    p->works.clear();
}

// Device address of this GPU's copy of `scratch`, looked up on the first call
// with that device current.
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

static dctplus_status scratch_ptr(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(DCTPLUS_EUNSUPPORTED, "device %d: at most %d devices", dev,
                                                   kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return e != hipSuccess ? hip_fail(e, "hipGetSymbolAddress(scratch)")
                                   : fail(DCTPLUS_EDEVICE, "no device address for the static scratch");
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return DCTPLUS_OK;
}

bool route_alloc_free(const dctplus_plan_s *p) {
    if (p->route == DCTPLUS_ROUTE_FAST) return fast_in_lds(p);
    // dense routes need a workspace only for the factored form above n = 64 (the DCT
    // pass writes its output there before the product)
    return p->t.folded || p->n <= 64;
}

static bool aligned(const void *ptr, size_t a) { return ((uintptr_t)ptr % a) == 0; }

static size_t elem_size(const dctplus_plan_s *p) { return p->dtype == DCTPLUS_F64 ? 8 : 4; }

static dctplus_status check_io(const dctplus_plan_s *p, const void *in, const void *out, int64_t batch) {
    if (!p) return fail(DCTPLUS_EINVAL, "null plan");
    if (batch < 0) return fail(DCTPLUS_EINVAL, "batch = %lld < 0", (long long)batch);
    if (batch == 0) return DCTPLUS_OK;
    if (!in || !out) return fail(DCTPLUS_EINVAL, "null signal pointer");
    const size_t es = elem_size(p);
    if (!aligned(in, es) || !aligned(out, es)) return fail(DCTPLUS_EINVAL, "misaligned signal pointer");
    const size_t bytes = (size_t)batch * p->n * es;
    const char *a = (const char *)in, *b = (const char *)out;
    if (a < b + bytes && b < a + bytes) return fail(DCTPLUS_EINVAL, "input and output overlap");
    if ((uint64_t)batch > (uint64_t)INT64_MAX / (uint64_t)p->n / es)
        return fail(DCTPLUS_EINVAL, "batch too large");
    return DCTPLUS_OK;
}

static dctplus_status set_device(const dctplus_plan_s *p) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (cur != p->device) {
        e = hipSetDevice(p->device);
        if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    }
    return DCTPLUS_OK;
}

// ---------------------------------------------------------------------------
// Tuning cache: a flat JSON object {"<key>": <config id>, ...}, one entry per line, keyed
// by device architecture, n, route, dtype, form, direction and batch bucket.
// ---------------------------------------------------------------------------
static std::string tune_prefix(const dctplus_plan_s *p) {
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t colon = arch.find(':');
        if (colon != std::string::npos) arch = arch.substr(0, colon);
    }
    char buf[192];
    // fast_below: batches below it run the FAST route on an AUTO plan kept on the dense
    // product, so its small-batch entries are FAST launch choices
    snprintf(buf, sizeof(buf), "%s|n=%lld|route=%d|dtype=%d|factored=%d|folded=%d|fast_below=%lld|", arch.c_str(),
             (long long)p->n, p->route, p->dtype, p->factored, p->t.folded, (long long)p->auto_fast_below);
    return buf;
}

static std::map<std::string, int> cache_read(const char *path) {
    std::map<std::string, int> m;
    FILE *f = fopen(path, "r");
    if (!f) return m;
    char line[512];
    while (fgets(line, sizeof(line), f)) {
        const char *a = strchr(line, '"');
        if (!a) continue;
        const char *b = strchr(a + 1, '"');
        if (!b) continue;
        const char *c = strchr(b, ':');
        if (!c) continue;
        m[std::string(a + 1, b)] = atoi(c + 1);
    }
    fclose(f);
    return m;
}

static bool cache_write(const char *path, const std::map<std::string, int> &m) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return false;
    fprintf(f, "{\n");
    size_t i = 0;
    for (const auto &kv : m) fprintf(f, "  \"%s\": %d%s\n", kv.first.c_str(), kv.second, ++i < m.size() ? "," : "");
    fprintf(f, "}\n");
    const bool ok = fclose(f) == 0;
    return ok && rename(tmp.c_str(), path) == 0;
}

// Entries of the cache named by DCTPLUS_TUNE_CACHE that match this plan.
static void cache_apply(dctplus_plan_s *p) {
    const char *path = getenv("DCTPLUS_TUNE_CACHE");
    if (!path || !*path) return;
    const std::string pre = tune_prefix(p);
    for (const auto &kv : cache_read(path)) {
        if (kv.first.compare(0, pre.size(), pre) != 0) continue;
        int dir = -1, bucket = -1;
        if (sscanf(kv.first.c_str() + pre.size(), "dir=%d|bucket=%d", &dir, &bucket) != 2) continue;
        if (dir < 0 || dir > 1 || bucket < 0 || bucket > 63 || kv.second < 0 || kv.second > 8) continue;
        p->tune_cfg[dir][bucket] = (int8_t)kv.second;
    }
}

}  // namespace dctplus

using namespace dctplus;

extern "C" {

void dctplus_default_opts(dctplus_opts *o) {
    if (!o) return;
    o->dtype = DCTPLUS_F32;
    o->route = DCTPLUS_ROUTE_AUTO;
    o->defl_tol = 1e-13;
    o->nufft_width = 0;   // chosen per dtype at plan time
    o->direct_kappa = 0.0;   // chosen per dtype at plan time
    o->device = -1;
    o->factored = 0;
}

// Plans of dctplus_plan (k = 1) and dctplus_plan_rank_k: rho[k], V[k * n] on the host.
static dctplus_status plan_create(int64_t n, int32_t k, const double *rhos, const double *V, const dctplus_opts *opts,
                                  void *stream, dctplus_plan_t *out) {
    if (!out) return fail(DCTPLUS_EINVAL, "null output pointer");
    *out = nullptr;
    if (n < 2) return fail(DCTPLUS_EINVAL, "n = %lld < 2", (long long)n);
    if (k < 1 || k > kMaxRank) return fail(DCTPLUS_EINVAL, "k = %d: 1 <= k <= %d updates", (int)k, kMaxRank);
    if (n < 4 || n > 16384 || (n & (n - 1)))
        return fail(DCTPLUS_EUNSUPPORTED, "n = %lld: supported sizes are powers of two in [4, 16384]",
                    (long long)n);
    if (k > 1 && n > 4096)
        return fail(DCTPLUS_EUNSUPPORTED, "rank-k plans support n <= 4096 (dense n x n FP64 set-up)");
    if (!rhos) return fail(DCTPLUS_EINVAL, "null rho");
    if (!V) return fail(DCTPLUS_EINVAL, "null v");
    for (int j = 0; j < k; ++j) {
        if (!isfinite(rhos[j])) return fail(DCTPLUS_EINVAL, "rho[%d] is not finite", j);
        for (int64_t i = 0; i < n; ++i)
            if (!isfinite(V[(size_t)j * n + i]))
                return fail(DCTPLUS_EINVAL, "v[%d][%lld] is not finite", j, (long long)i);
    }
    const double rho = rhos[0];
    const double *v_host = V;
    dctplus_opts o;
    dctplus_default_opts(&o);
    if (opts) o = *opts;
    if (o.dtype < DCTPLUS_F32 || o.dtype > DCTPLUS_F32_SPLIT) return fail(DCTPLUS_EINVAL, "bad dtype %d", o.dtype);
    if (o.route < DCTPLUS_ROUTE_AUTO || o.route > DCTPLUS_ROUTE_GFT)
        return fail(DCTPLUS_EINVAL, "bad route %d", o.route);
    if (!(o.defl_tol > 0.0)) o.defl_tol = 1e-13;
    // exact-row threshold on the NUFFT error amplification: 1e5 keeps FP32 plans within
    // 1e-6; FP64 plans take rows amplifying the window error by more than 1e3 exactly
    if (!(o.direct_kappa > 0.0)) o.direct_kappa = (o.dtype == DCTPLUS_F64) ? 1e3 : 1e5;
    // window taps: 12 reach the FP32 bar, FP64 plans need 16 (error ~1e-14)
    if (o.nufft_width == 0) o.nufft_width = (o.dtype == DCTPLUS_F64) ? 16 : 12;
    if (o.nufft_width < 4 || o.nufft_width > kMaxWidth || (o.nufft_width & 1))
        return fail(DCTPLUS_EINVAL, "nufft_width %d: must be even, 4..%d", o.nufft_width, kMaxWidth);
    int route = o.route;
    if (k > 1) {
        // later updates have non-Chebyshev poles: the composite factor is applied densely
        if (route == DCTPLUS_ROUTE_FAST)
            return fail(DCTPLUS_EUNSUPPORTED, "rank-k plans (k > 1) use the DENSE and GFT routes");
        if (route == DCTPLUS_ROUTE_AUTO) route = DCTPLUS_ROUTE_DENSE;
    }
    if (route == DCTPLUS_ROUTE_AUTO) {
        // measured on MI355X (forward + adjoint, FP32, 256 to 16,384 signals): the O(n^2)
        // MFMA product wins up to n = 512 at every batch and at n = 1024 from 4,096
        // signals on; the O(n log n) route wins from n = 2048 on at every batch (1.2-1.8x
        // at n = 2048, 1.9-2.7x at n = 4096).  FP64 plans stay on the dense product, which
        // is exact to 1e-12 (the FAST route to ~1e-11, its window error)
        route = (n >= 2048 && o.dtype == DCTPLUS_F32) ? DCTPLUS_ROUTE_FAST : DCTPLUS_ROUTE_DENSE;
    }
    if ((o.dtype == DCTPLUS_BF16 || o.dtype == DCTPLUS_F32_SPLIT) && route == DCTPLUS_ROUTE_FAST)
        return fail(DCTPLUS_EUNSUPPORTED, "BF16 operands apply to the DENSE and GFT routes");
    if (o.dtype == DCTPLUS_F32_SPLIT && (n < 32 || n > 4096))
        return fail(DCTPLUS_EUNSUPPORTED, "the split-BF16 mode supports 32 <= n <= 4096");
    if (o.dtype == DCTPLUS_F32_SPLIT && o.factored == 1 && n != 64)
        return fail(DCTPLUS_EUNSUPPORTED, "the factored split-BF16 form supports n = 64");

    if (o.dtype == DCTPLUS_BF16 && (n < 32 || n > 64))
        return fail(DCTPLUS_EUNSUPPORTED, "BF16 dense routes support n in {32, 64}");
    if (o.factored != 0 && o.factored != 1) return fail(DCTPLUS_EINVAL, "factored must be 0 or 1");
    if (o.factored && (route != DCTPLUS_ROUTE_DENSE ||
                       (o.dtype != DCTPLUS_F32 && o.dtype != DCTPLUS_BF16 && o.dtype != DCTPLUS_F32_SPLIT)))
        return fail(DCTPLUS_EUNSUPPORTED,
                    "the factored form is available on the DENSE route for F32, BF16 and F32_SPLIT");

    int dev = o.device;
    hipError_t e;
    if (dev < 0) {
        if ((e = hipGetDevice(&dev)) != hipSuccess) return hip_fail(e, "hipGetDevice");
    } else if ((e = hipSetDevice(dev)) != hipSuccess) {
        return hip_fail(e, "hipSetDevice");
    }
    dctplus_plan_s *p = new (std::nothrow) dctplus_plan_s();
    if (!p) return fail(DCTPLUS_ENOMEM, "host allocation failed");
    p->n = n;
    p->logn = 0;
    while ((1LL << p->logn) < n) ++p->logn;
    p->rho = rho;
    p->dtype = o.dtype;
    p->route = route;
    p->device = dev;
    p->defl_tol = o.defl_tol;
    p->direct_kappa = o.direct_kappa;
    p->width = o.nufft_width;
    p->factored = o.factored;
    p->rank = k;
    p->defer_dense = (k > 1);
    dctplus_status st = plan_build(p, v_host, (hipStream_t)stream);
    if (st == DCTPLUS_OK && k > 1) st = rank_k_build(p, k, rhos, V, (hipStream_t)stream);
    if (st != DCTPLUS_OK) {
        dctplus_plan_destroy(p);
        return st;
    }
    // AUTO at n = 1024 (FP32, one update): the dense product wins from about a thousand
    // signals on, the O(n log n) route below (measured forward + adjoint, 256 signals:
    // 0.047 against 0.064 ms; 512: 0.057 against 0.062); the FAST tables are built for
    // every plan, so small batches take that route per call
    if (o.route == DCTPLUS_ROUTE_AUTO && route == DCTPLUS_ROUTE_DENSE && k == 1 && n == 1024 &&
        o.dtype == DCTPLUS_F32 && !o.factored && p->t.ndirect <= kMaxDirect)
        p->auto_fast_below = 1024;
    cache_apply(p);
    *out = p;
    return DCTPLUS_OK;
}

dctplus_status dctplus_plan(int64_t n, double rho, const double *v_host, const dctplus_opts *opts, void *stream,
                            dctplus_plan_t *out) {
    return plan_create(n, 1, &rho, v_host, opts, stream, out);
}

dctplus_status dctplus_plan_rank_k(int64_t n, int32_t k, const double *rho_host, const double *V_host,
                                   const dctplus_opts *opts, void *stream, dctplus_plan_t *out) {
    return plan_create(n, k, rho_host, V_host, opts, stream, out);
}

dctplus_status dctplus_plan_general(int64_t n, const double *lambda_host, const double *U_host, double rho,
                                    const double *v_host, const dctplus_opts *opts, void *stream,
                                    dctplus_plan_t *out) {
    if (!out) return fail(DCTPLUS_EINVAL, "null output pointer");
    *out = nullptr;
    if (n < 2) return fail(DCTPLUS_EINVAL, "n = %lld < 2", (long long)n);
    if (n < 4 || n > 4096 || (n & (n - 1)))
        return fail(DCTPLUS_EUNSUPPORTED, "n = %lld: general-base plans support powers of two in [4, 4096]",
                    (long long)n);
    if (!lambda_host || !U_host || !v_host) return fail(DCTPLUS_EINVAL, "null lambda, U or v");
    if (!isfinite(rho)) return fail(DCTPLUS_EINVAL, "rho is not finite");
    for (int64_t i = 0; i < n; ++i) {
        if (!isfinite(lambda_host[i]) || !isfinite(v_host[i]))
            return fail(DCTPLUS_EINVAL, "lambda[%lld] or v[%lld] is not finite", (long long)i, (long long)i);
        if (i > 0 && !(lambda_host[i] > lambda_host[i - 1]))
            return fail(DCTPLUS_EINVAL, "lambda must be strictly increasing (index %lld)", (long long)i);
    }
    for (int64_t i = 0; i < n * n; ++i)
        if (!isfinite(U_host[i])) return fail(DCTPLUS_EINVAL, "U has a non-finite entry");
    dctplus_opts o;
    dctplus_default_opts(&o);
    if (opts) o = *opts;
    if (o.dtype < DCTPLUS_F32 || o.dtype > DCTPLUS_F32_SPLIT) return fail(DCTPLUS_EINVAL, "bad dtype %d", o.dtype);
    if (o.route < DCTPLUS_ROUTE_AUTO || o.route > DCTPLUS_ROUTE_GFT)
        return fail(DCTPLUS_EINVAL, "bad route %d", o.route);
    if (o.route == DCTPLUS_ROUTE_FAST || o.factored)
        return fail(DCTPLUS_EUNSUPPORTED, "a general base has no fast transform here: its plans apply the dense "
                                          "product with X^T (DENSE, GFT or AUTO, not factored)");
    if (o.dtype == DCTPLUS_BF16 && (n < 32 || n > 64))
        return fail(DCTPLUS_EUNSUPPORTED, "BF16 operands support n in {32, 64}");
    if (o.dtype == DCTPLUS_F32_SPLIT && (n < 32 || n > 4096))
        return fail(DCTPLUS_EUNSUPPORTED, "the split-BF16 mode supports 32 <= n <= 4096");
    if (!(o.defl_tol > 0.0)) o.defl_tol = 1e-13;
    int dev = o.device;
    hipError_t e;
    if (dev < 0) {
        if ((e = hipGetDevice(&dev)) != hipSuccess) return hip_fail(e, "hipGetDevice");
    } else if ((e = hipSetDevice(dev)) != hipSuccess) {
        return hip_fail(e, "hipSetDevice");
    }
    dctplus_plan_s *p = new (std::nothrow) dctplus_plan_s();
    if (!p) return fail(DCTPLUS_ENOMEM, "host allocation failed");
    p->n = n;
    p->logn = 0;
    while ((1LL << p->logn) < n) ++p->logn;
    p->rho = rho;
    p->dtype = o.dtype;
    p->route = DCTPLUS_ROUTE_GFT;   // the dense product with X^T
    p->device = dev;
    p->defl_tol = o.defl_tol;
    p->direct_kappa = 1e5;
    p->width = 12;
    p->factored = 0;
    p->rank = 1;
    p->general = 1;
    dctplus_status st = general_build(p, lambda_host, U_host, v_host, (hipStream_t)stream);
    if (st != DCTPLUS_OK) {
        dctplus_plan_destroy(p);
        return st;
    }
    cache_apply(p);
    *out = p;
    return DCTPLUS_OK;
}

dctplus_status dctplus_forward(dctplus_plan_t p, const void *x, void *y, int64_t batch, void *stream) {
    dctplus_status st = check_io(p, x, y, batch);
    if (st != DCTPLUS_OK || batch == 0) return st;
    if ((st = set_device(p)) != DCTPLUS_OK) return st;
    if (use_fast(p, batch)) return fast_apply(p, x, y, batch, false, (hipStream_t)stream);
    return dense_apply(p, x, y, batch, false, (hipStream_t)stream);
}

dctplus_status dctplus_adjoint(dctplus_plan_t p, const void *y, void *x, int64_t batch, void *stream) {
    dctplus_status st = check_io(p, y, x, batch);
    if (st != DCTPLUS_OK || batch == 0) return st;
    if ((st = set_device(p)) != DCTPLUS_OK) return st;
    if (use_fast(p, batch)) return fast_apply(p, y, x, batch, true, (hipStream_t)stream);
    return dense_apply(p, y, x, batch, true, (hipStream_t)stream);
}

dctplus_status dctplus_grad(dctplus_plan_t p, const void *y, const void *gy, int64_t batch, void *gx, double *grho,
                            double *gv, void *stream) {
    if (!p) return fail(DCTPLUS_EINVAL, "null plan");
    if ((p->rank > 1 || p->general) && (grho || gv))
        return fail(DCTPLUS_EUNSUPPORTED, "d/drho and d/dv are implemented for rank-one updates of the path");
    if (p->dtype != DCTPLUS_F32 && p->dtype != DCTPLUS_F32_SPLIT)
        return fail(DCTPLUS_EUNSUPPORTED, "gradients are implemented for FP32 plans");
    if (batch < 0) return fail(DCTPLUS_EINVAL, "batch = %lld < 0", (long long)batch);
    if (!y || !gy) return fail(DCTPLUS_EINVAL, "null y or gy");
    if (!aligned(y, 4) || !aligned(gy, 4) || (gx && !aligned(gx, 4)) || (grho && !aligned(grho, 8)) ||
        (gv && !aligned(gv, 8)))
        return fail(DCTPLUS_EINVAL, "misaligned pointer");
    if (gx) {
        dctplus_status st = check_io(p, gy, gx, batch);
        if (st != DCTPLUS_OK) return st;
    }
    dctplus_status st = set_device(p);
    if (st != DCTPLUS_OK) return st;
    return grad_apply(p, (const float *)y, (const float *)gy, batch, (float *)gx, grho, gv, (hipStream_t)stream);
}

dctplus_status dctplus_grad_noalloc(dctplus_plan_t p, const void *y, const void *gy, int64_t batch, void *gx,
                                    double *grho, double *gv, void *stream) {
    if (!p) return fail(DCTPLUS_EINVAL, "null plan");
    if ((p->rank > 1 || p->general) && (grho || gv))
        return fail(DCTPLUS_EUNSUPPORTED, "d/drho and d/dv are implemented for rank-one updates of the path");
    if (p->dtype != DCTPLUS_F32 && p->dtype != DCTPLUS_F32_SPLIT)
        return fail(DCTPLUS_EUNSUPPORTED, "gradients are implemented for FP32 plans");
    if (batch < 0) return fail(DCTPLUS_EINVAL, "batch = %lld < 0", (long long)batch);
    if (!y || !gy) return fail(DCTPLUS_EINVAL, "null y or gy");
    if (!aligned(y, 4) || !aligned(gy, 4) || (gx && !aligned(gx, 4)) || (grho && !aligned(grho, 8)) ||
        (gv && !aligned(gv, 8)))
        return fail(DCTPLUS_EINVAL, "misaligned pointer");
    if (gx) {
        dctplus_status st = check_io(p, gy, gx, batch);
        if (st != DCTPLUS_OK) return st;
    }
    dctplus_status st = set_device(p);
    if (st != DCTPLUS_OK) return st;
    void *ptr = nullptr;
    if ((st = scratch_ptr(p->device, &ptr)) != DCTPLUS_OK) return st;
    return grad_apply_static(p, (const float *)y, (const float *)gy, batch, (float *)gx, grho, gv, ptr,
                             kStaticScratchBytes, (hipStream_t)stream);
}

dctplus_status dctplus_tune(dctplus_plan_t p, void *x, void *y, int64_t batch, void *stream, const char *cache_path,
                            int32_t *chosen, float *ms) {
    dctplus_status st = check_io(p, x, y, batch);
    if (st != DCTPLUS_OK) return st;
    if (batch == 0) return fail(DCTPLUS_EINVAL, "batch = 0: nothing to time");
    if ((st = set_device(p)) != DCTPLUS_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const int count = use_fast(p, batch) ? fast_tune_count(p) : dense_tune_count(p, batch);
    const int b = batch_bucket(batch);
    if (ms)
        for (int i = 0; i < 16; ++i) ms[i] = 0.0f;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e;
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return hip_fail(e, "tuner events");
    }
    int best[2] = {0, 0};
    for (int dir = 0; dir < 2 && st == DCTPLUS_OK; ++dir) {
        const bool adj = dir == 1;
        float best_ms = 0.0f;
        for (int c = 1; c <= count && count > 1 && st == DCTPLUS_OK; ++c) {
            p->tune_cfg[dir][b] = (int8_t)c;
            auto call = [&]() {
                return adj ? dctplus_adjoint(p, y, x, batch, stream) : dctplus_forward(p, x, y, batch, stream);
            };
            if ((st = call()) != DCTPLUS_OK) break;                      // warm-up
            if ((e = hipEventRecord(e0, s)) != hipSuccess) { st = hip_fail(e, "tuner event"); break; }
            for (int r = 0; r < 3 && st == DCTPLUS_OK; ++r) st = call();
            if (st != DCTPLUS_OK) break;
            float t = 0.0f;
            if ((e = hipEventRecord(e1, s)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess ||
                (e = hipEventElapsedTime(&t, e0, e1)) != hipSuccess) {
                st = hip_fail(e, "tuner timing");
                break;
            }
            t /= 3.0f;
            if (ms && c <= 8) ms[8 * dir + c - 1] = t;
            if (best[dir] == 0 || t < best_ms) {
                best[dir] = c;
                best_ms = t;
            }
        }
        p->tune_cfg[dir][b] = (int8_t)best[dir];
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != DCTPLUS_OK) {
        p->tune_cfg[0][b] = p->tune_cfg[1][b] = 0;
        return st;
    }
    if (chosen) {
        chosen[0] = best[0];
        chosen[1] = best[1];
    }
    if (cache_path && *cache_path && count > 1) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);   // serialises writers in this process
        auto m = cache_read(cache_path);
        const std::string pre = tune_prefix(p);
        for (int dir = 0; dir < 2; ++dir) {
            char k[64];
            snprintf(k, sizeof(k), "dir=%d|bucket=%d", dir, b);
            m[pre + k] = best[dir];
        }
        if (!cache_write(cache_path, m)) return fail(DCTPLUS_EINVAL, "cannot write the tuning cache %s", cache_path);
    }
    return DCTPLUS_OK;
}

dctplus_status dctplus_plan_info(dctplus_plan_t p, double *mu, double *a, double *z, int32_t *kind,
                                 int32_t *counts) {
    if (!p) return fail(DCTPLUS_EINVAL, "null plan");
    dctplus_status st = set_device(p);
    if (st != DCTPLUS_OK) return st;
    const size_t nd = sizeof(double) * p->n;
    hipError_t e = hipSuccess;
    if (mu && (e = hipMemcpy(mu, p->t.mu, nd, hipMemcpyDeviceToHost)) != hipSuccess) return hip_fail(e, "info mu");
    if (a && (e = hipMemcpy(a, p->t.a, nd, hipMemcpyDeviceToHost)) != hipSuccess) return hip_fail(e, "info a");
    if (z && (e = hipMemcpy(z, p->t.z, nd, hipMemcpyDeviceToHost)) != hipSuccess) return hip_fail(e, "info z");
    if (kind && (e = hipMemcpy(kind, p->t.kind, sizeof(int32_t) * p->n, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "info kind");
    if (counts) {
        counts[0] = p->t.ndefl;
        counts[1] = p->t.ndirect;
        counts[2] = p->t.width;
        counts[3] = p->route;
    }
    return DCTPLUS_OK;
}

dctplus_status dctplus_plan_table(dctplus_plan_t p, const char *name, void *dst, int64_t *bytes) {
    if (!p || !name || !bytes) return fail(DCTPLUS_EINVAL, "null argument");
    const int64_t n = p->n, w = p->t.width, nd = p->t.ndirect;
    struct Entry { const char *name; const void *ptr; int64_t size; };
    const Entry tab[] = {
        {"z", p->t.z, 8 * n}, {"zraw", p->t.zraw, 8 * n}, {"mu", p->t.mu, 8 * n}, {"a", p->t.a, 8 * n},
        {"tau", p->t.tau, 8 * n}, {"hz", p->t.hz, 8 * n}, {"deconv", p->t.deconv, 8 * n},
        {"rowA", p->t.rowA, 8 * n}, {"rowB", p->t.rowB, 8 * n}, {"win", p->t.win, 8 * n * w},
        {"wina", p->t.wina, 8 * n * kTaps}, {"wspr", p->t.wspr, 8 * 2 * n * kReach},
        {"direct", p->t.direct, 8 * n * (nd <= kMaxDirect ? nd : 0)}, {"sintab", p->t.sintab, 8 * (2 * n + 1)},
        {"origin", p->t.origin, 4 * n}, {"kind", p->t.kind, 4 * n}, {"ref", p->t.ref, 4 * n},
        {"m0", p->t.m0, 4 * n}, {"rowOfBin", p->t.rowOfBin, 4 * n}, {"rowOfK", p->t.rowOfK, 4 * n},
        {"direct_row", p->t.direct_row, 4 * (nd < kMaxDirect ? nd : kMaxDirect)},
        {"ntie", p->t.status + 4, 4},
    };
    if (strcmp(name, "tune") == 0) {
        // host table: int8 [2 directions][64 batch buckets], the tuner's choices (0 = built-in)
        const int64_t cap = *bytes;
        *bytes = (int64_t)sizeof(p->tune_cfg);
        if (!dst) return DCTPLUS_OK;
        if (cap < *bytes) return fail(DCTPLUS_EINVAL, "buffer of %lld bytes is smaller than %lld", (long long)cap,
                                      (long long)*bytes);
        memcpy(dst, p->tune_cfg, sizeof(p->tune_cfg));
        return DCTPLUS_OK;
    }
    for (const Entry &e : tab) {
        if (strcmp(e.name, name) != 0) continue;
        const int64_t cap = *bytes;
        *bytes = e.size;
        if (!dst || e.size == 0) return DCTPLUS_OK;
        if (cap < e.size) return fail(DCTPLUS_EINVAL, "buffer of %lld bytes is smaller than %lld", (long long)cap,
                                      (long long)e.size);
        dctplus_status st = set_device(p);
        if (st != DCTPLUS_OK) return st;
        hipError_t err = hipMemcpy(dst, e.ptr, (size_t)e.size, hipMemcpyDeviceToHost);
        if (err != hipSuccess) return hip_fail(err, "plan table copy");
        return DCTPLUS_OK;
    }
    return fail(DCTPLUS_EINVAL, "unknown table '%s'", name);
}

void dctplus_plan_destroy(dctplus_plan_t p) {
    if (!p) return;
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur != p->device) (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    if (p->t.direct) (void)hipFree(p->t.direct);
    if (p->t.direct32) (void)hipFree(p->t.direct32);
    if (p->t.mt32) (void)hipFree(p->t.mt32);
    if (p->t.mt16) (void)hipFree(p->t.mt16);
    if (p->t.mt64) (void)hipFree(p->t.mt64);
    dense_release(p);
    release_works(p);
    if (p->dev_mem) (void)hipFree(p->dev_mem);
    if (cur >= 0 && cur != p->device) (void)hipSetDevice(cur);
    delete p;
}

const char *dctplus_status_string(dctplus_status s) {
    switch (s) {
        case DCTPLUS_OK: return "ok";
        case DCTPLUS_EINVAL: return "invalid argument";
        case DCTPLUS_ENOMEM: return "out of memory";
        case DCTPLUS_EDEVICE: return "device error";
        case DCTPLUS_EUNSUPPORTED: return "unsupported";
        case DCTPLUS_ENOCONV: return "secular solver did not converge";
        case DCTPLUS_EDEGENERATE: return "double eigenvalue";
    }
    return "unknown status";
}

const char *dctplus_last_error(void) { return g_err; }

}  // extern "C"
