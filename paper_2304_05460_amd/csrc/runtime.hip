// Library runtime: error reporting, device memory bookkeeping, the per-device
// scratch area and the kernel_matvec entry point of the C-ABI.
#include <mutex>
#include <vector>
#include <string>

#include "afn_internal.h"

namespace afn {

// Below this size the ordering costs more than the pruning saves.
static constexpr int64_t kPruneMinN = 8192;
// Size of the static scratch array of kernel_matvec_noalloc (per device).
static constexpr size_t kStaticScratchBytes = (size_t)192 << 20;

static thread_local std::string g_last_error;

void set_error(const char *fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

void clear_error() { g_last_error.clear(); }

namespace {
struct PooledStream {
    int device;
    hipStream_t st;
    hipEvent_t ev0, ev1;
    bool busy;
};
// never destroyed: the thread's streams live until the process ends (their
// destruction at thread exit could run after the runtime's own teardown)
std::vector<PooledStream> &side_pool()
{
    static thread_local std::vector<PooledStream> *pool = new std::vector<PooledStream>();
    return *pool;
}
}  // namespace

afn_status SideStream::open()
{
    int dev = 0;
    AFN_HIP(hipGetDevice(&dev));
    auto &pool = side_pool();
    for (size_t i = 0; i < pool.size(); ++i)
        if (!pool[i].busy && pool[i].device == dev) {
            pool[i].busy = true;
            slot = (int)i;
            st = pool[i].st;
            ev0 = pool[i].ev0;
            ev1 = pool[i].ev1;
            return AFN_OK;
        }
    PooledStream e{dev, nullptr, nullptr, nullptr, true};
    AFN_HIP(hipStreamCreateWithFlags(&e.st, hipStreamNonBlocking));
    AFN_HIP(hipEventCreateWithFlags(&e.ev0, hipEventDisableTiming));
    AFN_HIP(hipEventCreateWithFlags(&e.ev1, hipEventDisableTiming));
    pool.push_back(e);
    slot = (int)pool.size() - 1;
    st = e.st;
    ev0 = e.ev0;
    ev1 = e.ev1;
    return AFN_OK;
}

SideStream::~SideStream()
{
    if (slot < 0) return;
    (void)hipStreamSynchronize(st);
    side_pool()[(size_t)slot].busy = false;
}

afn_status DevArena::alloc(void **p, size_t bytes)
{
    *p = nullptr;
    const size_t start = (size_t)round_up((int64_t)off, 256);
    if (!base || start + bytes > cap) {
        set_error("workspace exhausted: %zu bytes needed at offset %zu of %zu", bytes, start, cap);
        return AFN_ENOMEM;
    }
    *p = base + start;
    off = start + bytes;
    high = off > high ? off : high;
    return AFN_OK;
}

namespace {
struct Scratch {
    void *ptr = nullptr;
    size_t bytes = 0;
};
std::mutex g_scratch_mu;
Scratch g_scratch[64];
}  // namespace

afn_status library_scratch(size_t bytes, void **ptr)
{
    int dev = 0;
    AFN_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) {
        set_error("device ordinal %d out of range", dev);
        return AFN_EDEVICE;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    Scratch &sc = g_scratch[dev];
    if (sc.bytes < bytes) {
        if (sc.ptr) {
            AFN_HIP(hipDeviceSynchronize());
            AFN_HIP(hipFree(sc.ptr));
            sc.ptr = nullptr;
            sc.bytes = 0;
        }
        size_t want = bytes + bytes / 4;
        hipError_t e = hipMalloc(&sc.ptr, want);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            sc.ptr = nullptr;
            set_error("scratch hipMalloc(%zu) failed: %s", want, hipGetErrorString(e));
            return AFN_ENOMEM;
        }
        sc.bytes = want;
    }
    *ptr = sc.ptr;
    return AFN_OK;
}

}  // namespace afn

namespace afn {
namespace {

// Scratch of one kernel_matvec call, carved in this order: the spatial
// order's work area, the order itself, the packed points, the tile boxes and
// the partial sums (pruned path, d <= 8 and n >= kPruneMinN); packed points,
// column blocks and partials (many columns); partials only (plain path).
size_t kmv_call_scratch_bytes(int64_t n, int d, int nrhs)
{
    const int64_t npad = kmv_packed_doubles(n, d) / d;
    const int64_t R = nrhs >= 2 ? (nrhs < 64 ? nrhs : 64) : 0;
    if (d <= 8 && n >= kPruneMinN) {
        const size_t ob = round_up((int64_t)spatial_order_work_bytes(n, d), 256);
        const size_t pb = round_up(4 * n, 256);
        const size_t xb = round_up(8 * npad * d, 256);
        const size_t bb = round_up(8 * kmv_box_count(n, d), 256);
        const size_t wb = nrhs >= 2 ? sizeof(double) * (size_t)(2 * n * R + mrhs_part_elems(npad))
                                    : sizeof(double) * (size_t)kmv_workspace_doubles(n, d);
        return ob + pb + xb + bb + wb + 1024;
    }
    if (nrhs >= 2 && d <= 8)
        return sizeof(double) * (size_t)(npad * d + 2 * n * R + mrhs_part_elems(npad)) + 1024;
    return sizeof(double) * (size_t)kmv_workspace_doubles(n, d);
}

afn_status kmv_check_args(const char *who, const double *X_dev, int64_t n, int32_t d, double l, double mu,
                          const double *v_dev, double *y_dev, int32_t nrhs, int64_t ld, int32_t precision,
                          int32_t kind)
{
    if (n < 1 || d < 1 || d > kMaxD || !(l > 0) || !(mu >= 0) || nrhs < 1 || ld < n || !X_dev || !v_dev ||
        !y_dev) {
        set_error("%s: invalid argument (n=%lld d=%d l=%g mu=%g nrhs=%d ld=%lld)", who, (long long)n, d, l, mu,
                  nrhs, (long long)ld);
        return AFN_EINVAL;
    }
    if (precision != AFN_FP64 && precision != AFN_FP32) {
        set_error("%s: unknown precision %d", who, precision);
        return AFN_EINVAL;
    }
    if (kind != AFN_KERNEL_GAUSSIAN && kind != AFN_KERNEL_MATERN32) {
        set_error("%s: unknown kernel %d", who, kind);
        return AFN_EINVAL;
    }
    return AFN_OK;
}

// The body of kernel_matvec on a scratch area of kmv_call_scratch_bytes(n, d,
// nrhs) bytes at 'work' (256-byte aligned device memory).
afn_status kmv_call(const double *X_dev, int64_t n, int32_t d, double l, double mu, const double *v_dev,
                    double *y_dev, int32_t nrhs, int64_t ld, int32_t precision, int32_t kind, void *work,
                    hipStream_t s)
{
    if (d <= 8 && n >= kPruneMinN) {
        // spatial order, packed points and tile boxes: far-apart tile pairs are
        // skipped (kernel values below 2^-64 in FP64 tiles, 2^-44 in FP32)
        const bool f32 = precision == AFN_FP32;
        const int64_t npad = kmv_packed_doubles(n, d) / d;
        const int64_t R = nrhs >= 2 ? (nrhs < 64 ? nrhs : 64) : 0;
        const size_t ob = round_up((int64_t)spatial_order_work_bytes(n, d), 256);
        const size_t pb = round_up(4 * n, 256);
        const size_t xb = round_up(8 * npad * d, 256);
        const size_t bb = round_up(8 * kmv_box_count(n, d), 256);
        char *base = (char *)work;
        void *ows = base;
        int32_t *kperm = (int32_t *)(base + ob);
        void *Xs = base + ob + pb;
        void *box = base + ob + pb + xb;
        double *rest = (double *)(base + ob + pb + xb + bb);
        AFN_TRY(spatial_order(X_dev, n, d, kperm, ows, s));
        AFN_TRY(kmv_pack(X_dev, n, d, l, kind, Xs, f32, s, kperm));
        AFN_TRY(kmv_boxes(Xs, n, d, f32, box, s));
        if (nrhs >= 2) {
            double *Pr = rest;
            double *Yr = Pr + n * R;
            double *part = Yr + n * R;
            for (int64_t c0 = 0; c0 < nrhs; c0 += 64) {
                const int Rc = (int)(nrhs - c0 < 64 ? nrhs - c0 : 64);
                if (f32) {
                    AFN_TRY(gather_rows<float>(v_dev + c0 * ld, ld, nullptr, n, Rc, nullptr, (float *)Pr, s));
                    AFN_TRY(kmv_mrhs_run<float>((const float *)Xs, npad, n, d, mu, kind, (const float *)Pr, Rc,
                                                (float *)Yr, Rc, Rc, (float *)part, s, nullptr, nullptr, kperm,
                                                (const float *)box));
                    AFN_TRY(scatter_rows_f32((const float *)Yr, n, Rc, y_dev + c0 * ld, ld, s));
                } else {
                    AFN_TRY(gather_rows<double>(v_dev + c0 * ld, ld, nullptr, n, Rc, nullptr, Pr, s));
                    AFN_TRY(kmv_mrhs_run<double>((const double *)Xs, npad, n, d, mu, kind, Pr, Rc, Yr, Rc, Rc,
                                                 part, s, nullptr, nullptr, kperm, (const double *)box));
                    AFN_TRY(scatter_rows(Yr, nullptr, n, Rc, y_dev + c0 * ld, ld, s));
                }
            }
            return AFN_OK;
        }
        if (f32)
            return kmv_packed_f32_dvec((const float *)Xs, n, d, mu, kind, v_dev, ld, y_dev, ld, nrhs,
                                       (float *)rest, s, kperm, (const float *)box);
        return kmv_packed_f64((const double *)Xs, n, d, mu, kind, v_dev, ld, y_dev, ld, nrhs, rest, s, nullptr,
                              nullptr, kperm, (const double *)box);
    }
    if (nrhs >= 2 && d <= 8) {
        // many columns: MFMA tile kernel on point-major blocks of <= 64 columns
        const int64_t npad = kmv_packed_doubles(n, d) / d;
        const int64_t R = nrhs < 64 ? nrhs : 64;
        double *Xs = (double *)work;
        double *Pr = Xs + npad * d;
        double *Yr = Pr + n * R;
        double *part = Yr + n * R;
        AFN_TRY(kmv_pack(X_dev, n, d, l, kind, Xs, precision == AFN_FP32, s));
        for (int64_t c0 = 0; c0 < nrhs; c0 += 64) {
            const int Rc = (int)(nrhs - c0 < 64 ? nrhs - c0 : 64);
            if (precision == AFN_FP32) {
                AFN_TRY(gather_rows<float>(v_dev + c0 * ld, ld, nullptr, n, Rc, nullptr, (float *)Pr, s));
                AFN_TRY(kmv_mrhs_run<float>((const float *)Xs, npad, n, d, mu, kind, (const float *)Pr, Rc,
                                            (float *)Yr, Rc, Rc, (float *)part, s));
                AFN_TRY(scatter_rows_f32((const float *)Yr, n, Rc, y_dev + c0 * ld, ld, s));
            } else {
                AFN_TRY(gather_rows<double>(v_dev + c0 * ld, ld, nullptr, n, Rc, nullptr, Pr, s));
                AFN_TRY(kmv_mrhs_run<double>(Xs, npad, n, d, mu, kind, Pr, Rc, Yr, Rc, Rc, part, s));
                AFN_TRY(scatter_rows(Yr, nullptr, n, Rc, y_dev + c0 * ld, ld, s));
            }
        }
        return AFN_OK;
    }
    if (precision == AFN_FP32)
        return kmv_f32(X_dev, n, d, l, mu, kind, v_dev, ld, y_dev, ld, nrhs, work, s);
    return kmv_f64(X_dev, n, d, l, mu, kind, v_dev, ld, y_dev, ld, nrhs, (double *)work, s);
}

// Scratch of kernel_matvec_noalloc: one static array per device, its address
// taken once per device with that device current.
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_static_mu;
void *g_static_ptr[64];

afn_status static_scratch(void **ptr)
{
    int dev = 0;
    AFN_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) {
        set_error("device ordinal %d out of range", dev);
        return AFN_EDEVICE;
    }
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            set_error("hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
            return AFN_EDEVICE;
        }
        g_static_ptr[dev] = p;
    }
    *ptr = g_static_ptr[dev];
    return AFN_OK;
}

}  // namespace
}  // namespace afn

extern "C" {

const char *afn_status_string(afn_status s)
{
    switch (s) {
        case AFN_OK: return "AFN_OK";
        case AFN_EINVAL: return "AFN_EINVAL: invalid argument";
        case AFN_ENOMEM: return "AFN_ENOMEM: device allocation failed";
        case AFN_ENOTSPD: return "AFN_ENOTSPD: matrix not positive definite";
        case AFN_ENOCONV: return "AFN_ENOCONV: no convergence within maxit";
        case AFN_EBREAKDOWN: return "AFN_EBREAKDOWN: CG breakdown";
        case AFN_ESTAGNATION: return "AFN_ESTAGNATION: refinement stagnated";
        case AFN_EDEVICE: return "AFN_EDEVICE: HIP runtime error";
    }
    return "unknown afn_status";
}

const char *afn_last_error(void) { return afn::g_last_error.c_str(); }

afn_status kernel_matvec(const double *X_dev, int64_t n, int32_t d, double l, double mu,
                         const double *v_dev, double *y_dev, int32_t nrhs, int64_t ld,
                         int32_t precision, void *stream)
{
    return kernel_matvec_ex(X_dev, n, d, l, mu, v_dev, y_dev, nrhs, ld, precision, AFN_KERNEL_GAUSSIAN, stream);
}


afn_status kernel_matvec_ex(const double *X_dev, int64_t n, int32_t d, double l, double mu,
                            const double *v_dev, double *y_dev, int32_t nrhs, int64_t ld,
                            int32_t precision, int32_t kind, void *stream)
{
    afn::clear_error();
    AFN_TRY(afn::kmv_check_args("kernel_matvec", X_dev, n, d, l, mu, v_dev, y_dev, nrhs, ld, precision, kind));
    void *work = nullptr;
    AFN_TRY(afn::library_scratch(afn::kmv_call_scratch_bytes(n, d, nrhs), &work));
    return afn::kmv_call(X_dev, n, d, l, mu, v_dev, y_dev, nrhs, ld, precision, kind, work, (hipStream_t)stream);
}

afn_status kernel_matvec_noalloc(const double *X_dev, int64_t n, int32_t d, double l, double mu,
                                 const double *v_dev, double *y_dev, int32_t nrhs, int64_t ld,
                                 int32_t precision, int32_t kind, void *stream)
{
    afn::clear_error();
    AFN_TRY(afn::kmv_check_args("kernel_matvec_noalloc", X_dev, n, d, l, mu, v_dev, y_dev, nrhs, ld, precision,
                                kind));
    const size_t need = afn::kmv_call_scratch_bytes(n, d, nrhs);
    if (need > afn::kStaticScratchBytes) {
        afn::set_error("kernel_matvec_noalloc: n=%lld d=%d nrhs=%d needs %zu bytes of scratch, more than the "
                       "%zu-byte static area",
                       (long long)n, d, nrhs, need, (size_t)afn::kStaticScratchBytes);
        return AFN_EINVAL;
    }
    void *work = nullptr;
    AFN_TRY(afn::static_scratch(&work));
    return afn::kmv_call(X_dev, n, d, l, mu, v_dev, y_dev, nrhs, ld, precision, kind, work, (hipStream_t)stream);
}

}  // extern "C"
