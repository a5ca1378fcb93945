// C ABI of the aperture-mass library (declared in include/amap.h): argument
// validation, contexts, device workspace, filter tables for the direct sum,
// and the sequencing of the kernels of each entry point.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "amap.h"
#include "amap_device.h"
#include "amap_launch.h"
#include "amap_host.h"

using namespace amap;

namespace {

thread_local std::string g_last_error;

amap_status fail(amap_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

amap_status hip_fail(hipError_t e, const char* what) {
    return fail(AMAP_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Makes the context's device current for the lifetime of the guard.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

bool is_pow2(long long v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(long long v) { int l = 0; while ((1ll << l) < v) ++l; return l; }

amap_status check_n(int n) {
    if (n < 16 || n > 4096 || !is_pow2(n))
        return fail(AMAP_E_INVAL, "n must be a power of two in [16, 4096] (got %d)", n);
    return AMAP_OK;
}
amap_status check_J(int n, int J) {
    if (J < 2) return fail(AMAP_E_INVAL, "J must be >= 2 (got %d)", J);
    if (J > 30 || (1ll << J) > n)
        return fail(AMAP_E_INVAL, "2^J must not exceed n (J=%d, n=%d)", J, n);
    return AMAP_OK;
}
amap_status check_ptr(const void* p, const char* name, bool required = true) {
    if (!p) return required ? fail(AMAP_E_INVAL, "%s must not be NULL", name) : AMAP_OK;
    if (reinterpret_cast<uintptr_t>(p) % 256 != 0)
        return fail(AMAP_E_INVAL, "%s must be 256-byte aligned", name);
    return AMAP_OK;
}
amap_status check_dtype(amap_dtype dt) {
    if (dt != AMAP_F32 && dt != AMAP_F64) return fail(AMAP_E_INVAL, "unknown dtype %d", (int)dt);
    return AMAP_OK;
}
bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    if (!a || !b) return false;
    const char* pa = static_cast<const char*>(a);
    const char* pb = static_cast<const char*>(b);
    return pa < pb + nb && pb < pa + na;
}
size_t esize(amap_dtype dt) { return dt == AMAP_F64 ? 8 : 4; }
size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

#define AMAP_TRY(expr)                           \
    do {                                         \
        amap_status s_ = (expr);                 \
        if (s_ != AMAP_OK) return s_;            \
    } while (0)
#define AMAP_HIP(expr, what)                     \
    do {                                         \
        hipError_t e_ = (expr);                  \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

}  // namespace

namespace amap {
KernelTimer*& current_timer() {
    static thread_local KernelTimer* t = nullptr;
    return t;
}
}  // namespace amap

// Per-kernel timing with HIP events recorded on each launch's stream.
struct EventTimer : KernelTimer {
    struct Rec {
        const char* name;
        hipEvent_t a, b;
    };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    std::map<std::string, std::pair<long long, double>> totals;  // launches, ms
    std::string only;  // time only launches of this name (empty: all)

    hipEvent_t get() {
        hipEvent_t e = nullptr;
        if (!pool.empty()) {
            e = pool.back();
            pool.pop_back();
        } else if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
        }
        return e;
    }
    void begin(const char* name, hipStream_t s) override {
        if (!only.empty() && only != name) {
            pending.push_back(Rec{name, nullptr, nullptr});
            return;
        }
        Rec r{name, get(), get()};
        if (r.a) (void)hipEventRecord(r.a, s);
        pending.push_back(r);
    }
    void end(hipStream_t s) override {
        if (!pending.empty() && pending.back().b) (void)hipEventRecord(pending.back().b, s);
    }
    void flush() {
        for (Rec& r : pending) {
            float ms = 0.f;
            if (r.a && r.b && hipEventSynchronize(r.b) == hipSuccess &&
                hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
                auto& t = totals[r.name];
                t.first += 1;
                t.second += ms;
            }
            if (r.a) pool.push_back(r.a);
            if (r.b) pool.push_back(r.b);
        }
        pending.clear();
    }
    ~EventTimer() override {
        flush();
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};

struct amap_ctx {
    int device = 0;
    cpx<float>* tw32 = nullptr;
    cpx<double>* tw64 = nullptr;
    Workspace ws;
    EventTimer* timer = nullptr;
    // tuned starlet schedules: (element size, log2 n, J, noise mode, batch) -> plan
    // (nstages == 0: the analytic planner)
    mutable std::map<std::array<int, 5>, StagePlan> plans;
    int autotune = 1;  // 0 analytic, 1 tuned, 2 analytic with sub-grid final noise stages
    mutable std::map<std::array<int, 5>, StagePlan> plans_sub;  // mode 2 schedules
    int noise_cap = 0;  // > 0: at most this many noise realisations per launch sequence
};

namespace {
// The tuned schedule for a starlet launch shaped like `a`, tuning it on a's
// buffers on first use (which overwrites a's outputs and, in noise mode, M
// and M2: callers tune before they zero the statistics).  Never tunes while
// the stream is being captured; then the analytic plan is used.
template <typename T>
const StagePlan* tuned_plan(const amap_ctx* c, const StarletArgs<T>& a) {
    if (c->autotune == 0) return nullptr;
    const std::array<int, 5> key{(int)sizeof(T), a.logn, a.J, a.M != nullptr, a.batch};
    if (c->autotune == 2) {
        if (!a.M) return nullptr;
        auto is = c->plans_sub.find(key);
        if (is != c->plans_sub.end()) return is->second.nstages ? &is->second : nullptr;
        StagePlan p;
        analytic_subgrid_plan<T>(1 << a.logn, a.J, &p);
        StagePlan& kept = (c->plans_sub[key] = p);
        return kept.nstages ? &kept : nullptr;
    }
    auto it = c->plans.find(key);
    if (it != c->plans.end()) return &it->second;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(a.stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
        (void)hipGetLastError();
        return nullptr;
    }
    StagePlan p;
    if (tune_starlet<T>(a, 3, &p) != hipSuccess) {
        (void)hipGetLastError();
        p.nstages = 0;
    }
    return &(c->plans[key] = p);
}
}  // namespace

namespace {
// Installs the context's timer (if any) for the calling thread.
struct TimerScope {
    KernelTimer* prev;
    explicit TimerScope(const amap_ctx* c) : prev(current_timer()) {
        current_timer() = c ? c->timer : nullptr;
    }
    ~TimerScope() { current_timer() = prev; }
};
}  // namespace

// ---- workspace ---------------------------------------------------------------------
amap_status Workspace::reserve(size_t bytes) {
    if (bytes <= size) return AMAP_OK;
    if (ptr) {
        // earlier work may still use the old buffer
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "device synchronize before workspace growth");
        (void)hipFree(ptr);
        ptr = nullptr;
        size = 0;
    }
    const size_t want = align256(bytes);
    if (hipMalloc(&ptr, want) != hipSuccess) {
        (void)hipGetLastError();
        ptr = nullptr;
        return fail(AMAP_E_NOMEM, "cannot allocate %zu bytes of device workspace", want);
    }
    size = want;
    return AMAP_OK;
}
void Workspace::release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    size = 0;
}

// ---- twiddles ----------------------------------------------------------------------
// exp(-2 pi i k / 4096), evaluated in long double and rounded once.
template <typename T>
static amap_status upload_twiddles(cpx<T>** out) {
    std::vector<T> host(2 * kMaxN);
    for (int k = 0; k < kMaxN; ++k) {
        const long double a = -2.0L * 3.14159265358979323846264338327950288L * k / kMaxN;
        host[2 * k] = (T)cosl(a);
        host[2 * k + 1] = (T)sinl(a);
    }
    void* p = nullptr;
    if (hipMalloc(&p, host.size() * sizeof(T)) != hipSuccess)
        return fail(AMAP_E_NOMEM, "cannot allocate twiddle table");
    if (hipMemcpy(p, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(p);
        return fail(AMAP_E_HIP, "cannot upload twiddle table");
    }
    *out = static_cast<cpx<T>*>(p);
    return AMAP_OK;
}

template <typename T> const cpx<T>* twiddles(const amap_ctx* c);
template <> const cpx<float>* twiddles<float>(const amap_ctx* c) { return c->tw32; }
template <> const cpx<double>* twiddles<double>(const amap_ctx* c) { return c->tw64; }

// ---- direct-sum tap table ----------------------------------------------------------------
static amap_status build_tap_table(amap_filter f, double theta, double fparam, double cut_px,
                                   int n, TapTable* t) {
    double cut = cut_px;
    if (!(cut > 0.0)) {
        cut = f == AMAP_FILTER_STARLET ? 2.0 * theta : (f == AMAP_FILTER_S98 ? theta : 5.0 * theta);
    }
    if (!std::isfinite(cut) || cut > 256.0)
        return fail(AMAP_E_INVAL, "cut radius %g exceeds the supported 256 px", cut);
    const int R = (int)std::floor(cut);
    if (2 * R + 1 > n)
        return fail(AMAP_E_INVAL, "cut radius %g too large for n = %d (need 2*floor(cut)+1 <= n)",
                    cut, n);
    const double c2 = cut * cut;
    const int D = 2 * R + 1;
    t->R = R;
    t->half.assign(D, -1);
    t->wc.assign((size_t)D * D, 0.0);
    t->ws.assign((size_t)D * D, 0.0);
    for (int dy = -R; dy <= R; ++dy) {
        for (int dx = -R; dx <= R; ++dx) {
            const double r2 = (double)(dx * dx + dy * dy);
            if (r2 > c2) continue;
            const int ax = dx < 0 ? -dx : dx;
            if (ax > t->half[dy + R]) t->half[dy + R] = ax;
            if (r2 == 0.0) continue;
            const double r = std::sqrt(r2);
            double q;
            if (f == AMAP_FILTER_STARLET) q = starlet_Q(r / theta) / (theta * theta);
            else if (f == AMAP_FILTER_S98) q = s98_Q(r, theta, fparam);
            else q = jbj04_Q(r, theta, fparam);
            const size_t i = (size_t)(dy + R) * D + (dx + R);
            t->wc[i] = q * (double)(dx * dx - dy * dy) / r2;
            t->ws[i] = q * 2.0 * (double)dx * (double)dy / r2;
        }
    }
    return AMAP_OK;
}

// ---- path pieces (typed) -------------------------------------------------------------
namespace amap {

template <typename T>
amap_status enqueue_ks(const amap_ctx* ctx, int logn, int batch, const T* g1, const T* g2,
                       long long g_stride, cpx<T>* C, T* kE, T* kB, long long out_stride,
                       bool rotate, uint64_t seed, uint64_t r0, hipStream_t s,
                       bool pair_e = false) {
    KsArgs<T> a;
    a.logn = logn; a.batch = batch; a.g1 = g1; a.g2 = g2; a.g_stride = g_stride; a.C = C;
    a.kE = kE; a.kB = kB; a.out_stride = out_stride; a.rotate = rotate; a.seed = seed;
    a.r0 = r0; a.tw = twiddles<T>(ctx); a.stream = s; a.pair_e = pair_e;
    AMAP_HIP(launch_ks<T>(a), "KS kernels");
    return AMAP_OK;
}

// Signal-path starlet: `scratch` holds 2*batch*n*n elements (c ping-pong
// buffer and the per-scale row-pass scratch).
template <typename T>
amap_status enqueue_starlet(const amap_ctx* ctx, int logn, int J, int batch, const T* kappa,
                            long long in_stride, T* planes, long long planes_stride, T* scratch,
                            hipStream_t s) {
    const long long n2 = 1ll << (2 * logn);
    StarletArgs<T> a;
    a.logn = logn; a.J = J; a.batch = batch; a.done = 0; a.kappa = kappa; a.in_stride = in_stride;
    a.planes = planes; a.planes_stride = planes_stride;
    a.cbuf0 = scratch; a.cbuf1 = nullptr; a.tmp = scratch + (long long)batch * n2; a.wbuf = nullptr;
    a.M = nullptr; a.M2 = nullptr; a.part = nullptr; a.stream = s;
    a.plan = tuned_plan<T>(ctx, a);
    AMAP_HIP(launch_starlet<T>(a), "starlet kernels");
    return AMAP_OK;
}

// Realisations per launch sequence of the noise loop.
int noise_batch(int n, int n_real) {
    const long long n2 = (long long)n * n;
    // ~128 M pixels of realisations in flight: fewer merges of the float64
    // running statistics (each reads and writes them once) and fewer launch
    // tails; 4.5 GiB of workspace at 1024^2
    long long b = (1ll << 27) / n2;
    if (b < 1) b = 1;
    if (b > n_real) b = n_real;
    return (int)b;
}

size_t noise_workspace_bytes(amap_dtype dt, int n, int J, int n_real) {
    const size_t n2 = (size_t)n * n, e = esize(dt);
    const size_t B = (size_t)noise_batch(n, n_real);
    return align256(B * n2 * 2 * e)            // complex spectra
         + 4 * align256(B * n2 * e)            // kappa, two c buffers, row scratch
         + align256(3 * B * n2 * e)            // detail planes of one stage
         + align256(starlet_partials_bytes(ilog2(n), (int)B))  // per-group partials
         + 2 * align256((size_t)(J - 1) * n2 * 8);  // running mean, M2
}

template <typename T>
amap_status enqueue_noise(const amap_ctx* ctx, char* ws, int n, int J, const T* g1,
                          const T* g2, int n_real, uint64_t seed, const T* planes_signal,
                          T* sigma, T* snr, hipStream_t s) {
    const int logn = ilog2(n);
    const long long n2 = (long long)n * n;
    // the workspace is sized for the default batch; a context's cap only
    // shrinks it
    int B = noise_batch(n, n_real);
    if (ctx->noise_cap > 0 && ctx->noise_cap < B) B = ctx->noise_cap;
    const size_t plane_b = align256((size_t)B * n2 * sizeof(T));
    char* p = ws;
    cpx<T>* C = reinterpret_cast<cpx<T>*>(p);   p += align256((size_t)B * n2 * 2 * sizeof(T));
    T* kap = reinterpret_cast<T*>(p);            p += plane_b;
    T* cb0 = reinterpret_cast<T*>(p);            p += plane_b;
    T* cb1 = reinterpret_cast<T*>(p);            p += plane_b;
    T* tmp = reinterpret_cast<T*>(p);            p += plane_b;
    T* wb = reinterpret_cast<T*>(p);             p += align256((size_t)3 * B * n2 * sizeof(T));
    void* part = p;                              p += align256(starlet_partials_bytes(logn, B));
    double* M = reinterpret_cast<double*>(p);    p += align256((size_t)(J - 1) * n2 * 8);
    double* M2 = reinterpret_cast<double*>(p);
    // the schedule of a full batch serves every batch; it is tuned (if new)
    // before the statistics are zeroed
    StarletArgs<T> t;
    t.logn = logn; t.J = J; t.batch = B; t.done = 0; t.kappa = kap; t.in_stride = n2;
    t.planes = nullptr; t.planes_stride = 0; t.cbuf0 = cb0; t.cbuf1 = cb1; t.tmp = tmp;
    t.wbuf = wb; t.M = M; t.M2 = M2; t.part = part; t.stream = s;
    const StagePlan* plan = tuned_plan<T>(ctx, t);
    // M and M2 need no clearing: the first batch's merges write them unread
    for (int r0 = 0; r0 < n_real; r0 += B) {
        const int bb = (n_real - r0) < B ? (n_real - r0) : B;
        AMAP_TRY(enqueue_ks<T>(ctx, logn, bb, g1, g2, 0, C, kap, nullptr, n2, true, seed,
                               (uint64_t)r0, s, /*pair_e=*/true));
        StarletArgs<T> a;
        a.logn = logn; a.J = J; a.batch = bb; a.done = r0; a.kappa = kap; a.in_stride = n2;
        a.planes = nullptr; a.planes_stride = 0; a.cbuf0 = cb0; a.cbuf1 = cb1; a.tmp = tmp;
        a.wbuf = wb; a.M = M; a.M2 = M2; a.part = part; a.stream = s; a.plan = plan;
        AMAP_HIP(launch_starlet<T>(a), "noise starlet kernels");
    }
    AMAP_HIP(launch_noise_finalize<T>(logn, J, n_real, M2, planes_signal, sigma, snr, s,
                                      stat_layout(plan)),
             "noise finalize");
    return AMAP_OK;
}

}  // namespace amap

// ---- static scratch of the no-allocation entry point ---------------------------------
// amap_ks_invert_noalloc takes its complex spectrum from this file-scope
// device array instead of the context's workspace.  Each GPU the library
// runs on holds its own copy until the process ends; host code reaches it
// only through the device address hipGetSymbolAddress returns (the array's
// name is a host-side stand-in, not a device address), looked up once per
// device when a context is created there.
constexpr size_t kNoAllocScratchBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;    // device -> address of its copy
std::map<int, std::string> g_scratch_err;

// With `device` current: look up and keep the device's scratch address.
void scratch_setup(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr.count(device)) return;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        g_scratch_err[device] = hipGetErrorString(e);
        return;
    }
    g_scratch_ptr[device] = ptr;
}

void* scratch_of(int device, std::string* why) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it != g_scratch_ptr.end()) return it->second;
    auto er = g_scratch_err.find(device);
    *why = er != g_scratch_err.end() ? er->second : "not set up on this device";
    return nullptr;
}
}  // namespace

// ---- C ABI -------------------------------------------------------------------------------
extern "C" {

const char* amap_last_error(void) { return g_last_error.c_str(); }

amap_status amap_create(int hip_device, amap_ctx_t* out) {
    g_last_error.clear();
    if (!out) return fail(AMAP_E_INVAL, "out must not be NULL");
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0)
        return fail(AMAP_E_HIP, "no HIP device available");
    if (hip_device < 0 || hip_device >= count)
        return fail(AMAP_E_INVAL, "device %d out of range (have %d)", hip_device, count);
    DeviceGuard g(hip_device);
    if (!g.ok) return fail(AMAP_E_HIP, "cannot select device %d", hip_device);
    amap_ctx* c = new (std::nothrow) amap_ctx;
    if (!c) return fail(AMAP_E_NOMEM, "out of host memory");
    c->device = hip_device;
    scratch_setup(hip_device);  // the no-allocation entry point's scratch on this device
    amap_status s = upload_twiddles<float>(&c->tw32);
    if (s == AMAP_OK) s = upload_twiddles<double>(&c->tw64);
    if (s != AMAP_OK) {
        if (c->tw32) (void)hipFree(c->tw32);
        delete c;
        return s;
    }
    *out = c;
    return AMAP_OK;
}

amap_status amap_destroy(amap_ctx_t c) {
    g_last_error.clear();
    if (!c) return AMAP_OK;
    DeviceGuard g(c->device);
    (void)hipDeviceSynchronize();
    delete c->timer;
    c->timer = nullptr;
    c->ws.release();
    if (c->tw32) (void)hipFree(c->tw32);
    if (c->tw64) (void)hipFree(c->tw64);
    delete c;
    return AMAP_OK;
}

amap_status amap_sync(amap_ctx_t c, void* stream) {
    g_last_error.clear();
    if (!c) return fail(AMAP_E_INVAL, "ctx must not be NULL");
    DeviceGuard g(c->device);
    AMAP_HIP(hipStreamSynchronize(static_cast<hipStream_t>(stream)), "stream synchronize");
    AMAP_HIP(hipGetLastError(), "asynchronous error");
    return AMAP_OK;
}

size_t amap_workspace_bytes(amap_ctx_t c) { return c ? c->ws.size : 0; }

amap_status amap_timing_enable(amap_ctx_t c, int enable) {
    g_last_error.clear();
    if (!c) return fail(AMAP_E_INVAL, "ctx must not be NULL");
    DeviceGuard g(c->device);
    if (enable && !c->timer) {
        c->timer = new (std::nothrow) EventTimer;
        if (!c->timer) return fail(AMAP_E_NOMEM, "out of host memory");
    } else if (!enable && c->timer) {
        delete c->timer;
        c->timer = nullptr;
    }
    return AMAP_OK;
}

// Reads the next integer after the quoted key (a key of amap_plans_read's
// format) at or after *p; advances *p past it.
static bool json_int(const char** p, const char* key, long* out) {
    const char* k = std::strstr(*p, key);
    if (!k) return false;
    const char* q = k + std::strlen(key);
    while (*q == ' ' || *q == ':' || *q == '"') ++q;
    char* end = nullptr;
    const long v = std::strtol(q, &end, 10);
    if (end == q) return false;
    *out = v;
    *p = end;
    return true;
}

amap_status amap_plans_load(amap_ctx_t c, const char* json) {
    g_last_error.clear();
    if (!c) return fail(AMAP_E_INVAL, "ctx must not be NULL");
    if (!json) return fail(AMAP_E_INVAL, "json must not be NULL");
    struct Entry { int mode; std::array<int, 5> key; StagePlan plan; };
    std::vector<Entry> got;
    const char* p = json;
    int idx = 0;
    while ((p = std::strchr(p, '{')) != nullptr) {
        long v[6];
        const char* keys[6] = {"\"mode\"", "\"elem\"", "\"logn\"", "\"J\"", "\"noise\"", "\"batch\""};
        for (int i = 0; i < 6; ++i)
            if (!json_int(&p, keys[i], &v[i])) return fail(AMAP_E_INVAL, "schedule %d: missing %s", idx, keys[i]);
        const char* st = std::strstr(p, "\"stages\"");
        if (!st) return fail(AMAP_E_INVAL, "schedule %d: missing \"stages\"", idx);
        st = std::strchr(st, '[');
        if (!st) return fail(AMAP_E_INVAL, "schedule %d: malformed stages", idx);
        ++st;
        Entry e;
        e.mode = (int)v[0];
        e.key = {(int)v[1], (int)v[2], (int)v[3], (int)v[4], (int)v[5]};
        e.plan.nstages = 0;
        // stages: [[j0, ns, tw, th, rb, kind], ...] up to the closing bracket
        while (true) {
            while (*st == ' ' || *st == ',') ++st;
            if (*st == ']') { ++st; break; }
            if (*st != '[' || e.plan.nstages >= 16) return fail(AMAP_E_INVAL, "schedule %d: malformed stages", idx);
            ++st;
            long f[6];
            for (int i = 0; i < 6; ++i) {
                while (*st == ' ' || *st == ',') ++st;
                char* end = nullptr;
                f[i] = std::strtol(st, &end, 10);
                if (end == st) return fail(AMAP_E_INVAL, "schedule %d: stage with fewer than 6 fields", idx);
                st = end;
            }
            while (*st == ' ') ++st;
            if (*st != ']') return fail(AMAP_E_INVAL, "schedule %d: stage with more than 6 fields", idx);
            ++st;
            e.plan.st[e.plan.nstages++] = StagePlan::Stage{(int)f[0], (int)f[1], (int)f[2], (int)f[3], (int)f[4], (int)f[5]};
        }
        p = st;
        const int elem = e.key[0], logn = e.key[1], J = e.key[2], noise = e.key[3], batch = e.key[4];
        if ((e.mode != 1 && e.mode != 2) || (elem != 4 && elem != 8) || logn < 4 || logn > kMaxLogN ||
            J < 2 || (1 << J) > (1 << logn) || (noise != 0 && noise != 1) || batch < 1)
            return fail(AMAP_E_INVAL, "schedule %d: bad mode, element size, size, J, noise flag or batch", idx);
        if (e.plan.nstages > 0) {
            const bool ok = elem == 4 ? plan_valid<float>(1 << logn, J, noise != 0, e.plan)
                                      : plan_valid<double>(1 << logn, J, noise != 0, e.plan);
            if (!ok) return fail(AMAP_E_INVAL, "schedule %d: not a valid stage schedule for n = %d, J = %d", idx, 1 << logn, J);
        }
        got.push_back(e);
        ++idx;
    }
    for (const Entry& e : got) (e.mode == 1 ? c->plans : c->plans_sub)[e.key] = e.plan;
    return AMAP_OK;
}

amap_status amap_plans_read(amap_ctx_t c, char* buf, size_t len) {
    g_last_error.clear();
    if (!c) return fail(AMAP_E_INVAL, "ctx must not be NULL");
    if (!buf || len == 0) return fail(AMAP_E_INVAL, "buf must not be NULL");
    std::string out = "[";
    bool first = true;
    for (int mode = 1; mode <= 2; ++mode) {
        for (const auto& kv : mode == 1 ? c->plans : c->plans_sub) {
            char item[192];
            snprintf(item, sizeof item, "%s{\"mode\": %d, \"elem\": %d, \"logn\": %d, \"J\": %d, \"noise\": %d, \"batch\": %d, \"stages\": [",
                     first ? "" : ", ", mode, kv.first[0], kv.first[1], kv.first[2], kv.first[3], kv.first[4]);
            out += item;
            for (int k = 0; k < kv.second.nstages; ++k) {
                const StagePlan::Stage& t = kv.second.st[k];
                snprintf(item, sizeof item, "%s[%d, %d, %d, %d, %d, %d]", k ? ", " : "", t.j0, t.ns, t.tw, t.th, t.rb, t.kind);
                out += item;
            }
            out += "]}";
            first = false;
        }
    }
    out += "]";
    if (out.size() + 1 > len) {
        buf[0] = 0;
        return fail(AMAP_E_INVAL, "buffer too small: need %zu bytes", out.size() + 1);
    }
    std::memcpy(buf, out.c_str(), out.size() + 1);
    return AMAP_OK;
}

amap_status amap_set_autotune(amap_ctx_t c, int enable) {
    g_last_error.clear();
    if (!c) return fail(AMAP_E_INVAL, "ctx must not be NULL");
    if (enable < 0 || enable > 2) return fail(AMAP_E_INVAL, "autotune mode must be 0, 1 or 2");
    c->autotune = enable;
    return AMAP_OK;
}

amap_status amap_set_noise_batch(amap_ctx_t c, int max_batch) {
    g_last_error.clear();
    if (!c) return fail(AMAP_E_INVAL, "ctx must not be NULL");
    if (max_batch < 0) return fail(AMAP_E_INVAL, "max_batch must be >= 0 (got %d)", max_batch);
    c->noise_cap = max_batch;
    return AMAP_OK;
}

amap_status amap_timing_select(amap_ctx_t c, const char* kernel) {
    g_last_error.clear();
    if (!c) return fail(AMAP_E_INVAL, "ctx must not be NULL");
    if (!c->timer) return fail(AMAP_E_INVAL, "timing is not enabled");
    DeviceGuard g(c->device);
    c->timer->flush();
    c->timer->only = kernel ? kernel : "";
    return AMAP_OK;
}

amap_status amap_timing_read(amap_ctx_t c, char* buf, size_t len, int reset) {
    g_last_error.clear();
    if (!c) return fail(AMAP_E_INVAL, "ctx must not be NULL");
    if (!buf || len == 0) return fail(AMAP_E_INVAL, "buf must not be NULL");
    std::string out = "{";
    if (c->timer) {
        DeviceGuard g(c->device);
        c->timer->flush();
        bool first = true;
        for (const auto& kv : c->timer->totals) {
            char item[256];
            snprintf(item, sizeof item, "%s\"%s\": [%lld, %.6f]", first ? "" : ", ",
                     kv.first.c_str(), kv.second.first, kv.second.second);
            out += item;
            first = false;
        }
        if (reset) c->timer->totals.clear();
    }
    out += "}";
    if (out.size() + 1 > len) {
        buf[0] = 0;
        return fail(AMAP_E_INVAL, "buffer too small: need %zu bytes", out.size() + 1);
    }
    std::memcpy(buf, out.c_str(), out.size() + 1);
    return AMAP_OK;
}

amap_status amap_ks_invert(amap_ctx_t c, amap_dtype dt, int n, const void* g1, const void* g2,
                           void* kappa_e, void* kappa_b, void* stream) {
    g_last_error.clear();
    if (!c) return fail(AMAP_E_INVAL, "ctx must not be NULL");
    AMAP_TRY(check_dtype(dt));
    AMAP_TRY(check_n(n));
    AMAP_TRY(check_ptr(g1, "g1"));
    AMAP_TRY(check_ptr(g2, "g2"));
    AMAP_TRY(check_ptr(kappa_e, "kappa_e"));
    AMAP_TRY(check_ptr(kappa_b, "kappa_b", false));
    const size_t bytes = (size_t)n * n * esize(dt);
    if (overlaps(kappa_e, bytes, g1, bytes) || overlaps(kappa_e, bytes, g2, bytes) ||
        overlaps(kappa_b, bytes, g1, bytes) || overlaps(kappa_b, bytes, g2, bytes) ||
        overlaps(kappa_e, bytes, kappa_b, bytes))
        return fail(AMAP_E_INVAL, "outputs may not overlap inputs or each other");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(AMAP_E_HIP, "cannot select device %d", c->device);
    TimerScope ts(c);
    AMAP_TRY(c->ws.reserve(2 * bytes));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int logn = ilog2(n);
    if (dt == AMAP_F32)
        return enqueue_ks<float>(c, logn, 1, (const float*)g1, (const float*)g2, 0,
                                 (cpx<float>*)c->ws.ptr, (float*)kappa_e, (float*)kappa_b,
                                 (long long)n * n, false, 0, 0, s);
    return enqueue_ks<double>(c, logn, 1, (const double*)g1, (const double*)g2, 0,
                              (cpx<double>*)c->ws.ptr, (double*)kappa_e, (double*)kappa_b,
                              (long long)n * n, false, 0, 0, s);
}

amap_status amap_ks_invert_noalloc(amap_ctx_t c, amap_dtype dt, int n, const void* g1,
                                   const void* g2, void* kappa_e, void* kappa_b, void* stream) {
    g_last_error.clear();
    if (!c) return fail(AMAP_E_INVAL, "ctx must not be NULL");
    AMAP_TRY(check_dtype(dt));
    AMAP_TRY(check_n(n));
    AMAP_TRY(check_ptr(g1, "g1"));
    AMAP_TRY(check_ptr(g2, "g2"));
    AMAP_TRY(check_ptr(kappa_e, "kappa_e"));
    AMAP_TRY(check_ptr(kappa_b, "kappa_b", false));
    const size_t bytes = (size_t)n * n * esize(dt);
    if (overlaps(kappa_e, bytes, g1, bytes) || overlaps(kappa_e, bytes, g2, bytes) ||
        overlaps(kappa_b, bytes, g1, bytes) || overlaps(kappa_b, bytes, g2, bytes) ||
        overlaps(kappa_e, bytes, kappa_b, bytes))
        return fail(AMAP_E_INVAL, "outputs may not overlap inputs or each other");
    if (2 * bytes > kNoAllocScratchBytes)
        return fail(AMAP_E_INVAL,
                    "n = %d needs %zu bytes of scratch; the no-allocation entry point holds %zu "
                    "(float32 and float64 up to n = 2048)", n, 2 * bytes, kNoAllocScratchBytes);
    std::string why;
    void* sp = scratch_of(c->device, &why);
    if (!sp) return fail(AMAP_E_HIP, "static scratch of device %d unavailable: %s", c->device, why.c_str());
    DeviceGuard g(c->device);
    if (!g.ok) return fail(AMAP_E_HIP, "cannot select device %d", c->device);
    TimerScope ts(c);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int logn = ilog2(n);
    if (dt == AMAP_F32)
        return enqueue_ks<float>(c, logn, 1, (const float*)g1, (const float*)g2, 0,
                                 static_cast<cpx<float>*>(sp), (float*)kappa_e, (float*)kappa_b,
                                 (long long)n * n, false, 0, 0, s);
    return enqueue_ks<double>(c, logn, 1, (const double*)g1, (const double*)g2, 0,
                              static_cast<cpx<double>*>(sp), (double*)kappa_e, (double*)kappa_b,
                              (long long)n * n, false, 0, 0, s);
}

amap_status amap_starlet_forward(amap_ctx_t c, amap_dtype dt, int n, int J, const void* kappa,
                                 void* planes, void* stream) {
    g_last_error.clear();
    if (!c) return fail(AMAP_E_INVAL, "ctx must not be NULL");
    AMAP_TRY(check_dtype(dt));
    AMAP_TRY(check_n(n));
    AMAP_TRY(check_J(n, J));
    AMAP_TRY(check_ptr(kappa, "kappa"));
    AMAP_TRY(check_ptr(planes, "planes"));
    const size_t plane = (size_t)n * n * esize(dt);
    if (overlaps(kappa, plane, planes, plane * J))
        return fail(AMAP_E_INVAL, "planes may not overlap kappa");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(AMAP_E_HIP, "cannot select device %d", c->device);
    TimerScope ts(c);
    AMAP_TRY(c->ws.reserve(2 * plane));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int logn = ilog2(n);
    const long long n2 = (long long)n * n;
    if (dt == AMAP_F32)
        return enqueue_starlet<float>(c, logn, J, 1, (const float*)kappa, n2, (float*)planes,
                                      (long long)J * n2, (float*)c->ws.ptr, s);
    return enqueue_starlet<double>(c, logn, J, 1, (const double*)kappa, n2, (double*)planes,
                                   (long long)J * n2, (double*)c->ws.ptr, s);
}

amap_status amap_starlet_forward_bc(amap_ctx_t c, amap_dtype dt, int ny, int nx, int J,
                                    int boundary, const void* image, void* planes, void* stream) {
    g_last_error.clear();
    if (!c) return fail(AMAP_E_INVAL, "ctx must not be NULL");
    AMAP_TRY(check_dtype(dt));
    if (ny < 2 || nx < 2 || ny > 16384 || nx > 16384)
        return fail(AMAP_E_INVAL, "field sides must be in [2, 16384] (got %d x %d)", ny, nx);
    if (J < 2 || J > 16) return fail(AMAP_E_INVAL, "J must be in [2, 16] (got %d)", J);
    if (boundary < AMAP_BC_PERIODIC || boundary > AMAP_BC_ZERO)
        return fail(AMAP_E_INVAL, "boundary must be AMAP_BC_PERIODIC, _MIRROR or _ZERO (got %d)", boundary);
    AMAP_TRY(check_ptr(image, "image"));
    AMAP_TRY(check_ptr(planes, "planes"));
    const size_t plane = (size_t)ny * nx * esize(dt);
    if (overlaps(image, plane, planes, plane * J))
        return fail(AMAP_E_INVAL, "planes may not overlap image");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(AMAP_E_HIP, "cannot select device %d", c->device);
    TimerScope ts(c);
    AMAP_TRY(c->ws.reserve(plane));
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (dt == AMAP_F32)
        AMAP_HIP(launch_starlet_bc<float>(ny, nx, J, boundary, (const float*)image, (float*)planes,
                                          (float*)c->ws.ptr, 1, 0, 0, s), "bounded starlet kernels");
    else
        AMAP_HIP(launch_starlet_bc<double>(ny, nx, J, boundary, (const double*)image, (double*)planes,
                                           (double*)c->ws.ptr, 1, 0, 0, s), "bounded starlet kernels");
    return AMAP_OK;
}

amap_status amap_ks_invert_padded(amap_ctx_t c, amap_dtype dt, int ny, int nx, int P,
                                  const void* g1, const void* g2, void* kappa_e, void* kappa_b,
                                  void* stream) {
    g_last_error.clear();
    if (!c) return fail(AMAP_E_INVAL, "ctx must not be NULL");
    AMAP_TRY(check_dtype(dt));
    AMAP_TRY(check_n(P));
    if (ny < 1 || nx < 1 || ny > P || nx > P)
        return fail(AMAP_E_INVAL, "field %d x %d must fit the %d x %d grid", ny, nx, P, P);
    AMAP_TRY(check_ptr(g1, "g1"));
    AMAP_TRY(check_ptr(g2, "g2"));
    AMAP_TRY(check_ptr(kappa_e, "kappa_e"));
    AMAP_TRY(check_ptr(kappa_b, "kappa_b", false));
    const size_t bytes = (size_t)ny * nx * esize(dt);
    if (overlaps(kappa_e, bytes, g1, bytes) || overlaps(kappa_e, bytes, g2, bytes) ||
        overlaps(kappa_b, bytes, g1, bytes) || overlaps(kappa_b, bytes, g2, bytes) ||
        overlaps(kappa_e, bytes, kappa_b, bytes))
        return fail(AMAP_E_INVAL, "outputs may not overlap inputs or each other");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(AMAP_E_HIP, "cannot select device %d", c->device);
    TimerScope ts(c);
    // workspace: complex spectrum (2 planes), padded g1, g2, kappa_E, kappa_B
    const size_t pb = align256((size_t)P * P * esize(dt));
    AMAP_TRY(c->ws.reserve(6 * pb));
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(c->ws.ptr);
    const int logn = ilog2(P);
    if (dt == AMAP_F32) {
        float *p1 = (float*)(w + 2 * pb), *p2 = (float*)(w + 3 * pb);
        float *e = (float*)(w + 4 * pb), *b = kappa_b ? (float*)(w + 5 * pb) : nullptr;
        AMAP_HIP(launch_pad2<float>((const float*)g1, (const float*)g2, ny, nx, P, p1, p2, s), "pad kernel");
        AMAP_TRY(enqueue_ks<float>(c, logn, 1, p1, p2, 0, (cpx<float>*)w, e, b, (long long)P * P,
                                   false, 0, 0, s));
        AMAP_HIP(launch_crop2<float>(e, b, P, ny, nx, (float*)kappa_e, (float*)kappa_b, 1, 0, 0, s),
                 "crop kernel");
    } else {
        double *p1 = (double*)(w + 2 * pb), *p2 = (double*)(w + 3 * pb);
        double *e = (double*)(w + 4 * pb), *b = kappa_b ? (double*)(w + 5 * pb) : nullptr;
        AMAP_HIP(launch_pad2<double>((const double*)g1, (const double*)g2, ny, nx, P, p1, p2, s),
                 "pad kernel");
        AMAP_TRY(enqueue_ks<double>(c, logn, 1, p1, p2, 0, (cpx<double>*)w, e, b, (long long)P * P,
                                    false, 0, 0, s));
        AMAP_HIP(launch_crop2<double>(e, b, P, ny, nx, (double*)kappa_e, (double*)kappa_b, 1, 0, 0, s),
                 "crop kernel");
    }
    return AMAP_OK;
}

static amap_status count_peaks_bc_impl(amap_ctx_t c, amap_dtype dt, int ny, int nx, int nplanes,
                                       int boundary, const void* planes, const unsigned char* mask,
                                       double threshold, long long* counts_dev, void* stream) {
    g_last_error.clear();
    if (!c) return fail(AMAP_E_INVAL, "ctx must not be NULL");
    AMAP_TRY(check_dtype(dt));
    if (ny < 2 || nx < 2 || ny > 16384 || nx > 16384)
        return fail(AMAP_E_INVAL, "plane sides must be in [2, 16384] (got %d x %d)", ny, nx);
    if (nplanes < 1 || nplanes > 65535)
        return fail(AMAP_E_INVAL, "nplanes must be in [1, 65535] (got %d)", nplanes);
    if (boundary < AMAP_BC_PERIODIC || boundary > AMAP_BC_ZERO)
        return fail(AMAP_E_INVAL, "boundary must be AMAP_BC_PERIODIC, _MIRROR or _ZERO (got %d)", boundary);
    AMAP_TRY(check_ptr(planes, "planes"));
    AMAP_TRY(check_ptr(counts_dev, "counts_dev"));
    AMAP_TRY(check_ptr(mask, "mask", false));
    DeviceGuard g(c->device);
    if (!g.ok) return fail(AMAP_E_HIP, "cannot select device %d", c->device);
    TimerScope ts(c);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (dt == AMAP_F32)
        AMAP_HIP(launch_count_peaks_bc<float>(ny, nx, nplanes, boundary, (const float*)planes, mask,
                                              threshold, counts_dev, s), "peak kernel");
    else
        AMAP_HIP(launch_count_peaks_bc<double>(ny, nx, nplanes, boundary, (const double*)planes, mask,
                                               threshold, counts_dev, s), "peak kernel");
    return AMAP_OK;
}

amap_status amap_count_peaks_bc(amap_ctx_t c, amap_dtype dt, int ny, int nx, int nplanes,
                                int boundary, const void* planes, double threshold,
                                long long* counts_dev, void* stream) {
    return count_peaks_bc_impl(c, dt, ny, nx, nplanes, boundary, planes, nullptr, threshold,
                               counts_dev, stream);
}

amap_status amap_count_peaks_masked(amap_ctx_t c, amap_dtype dt, int ny, int nx, int nplanes,
                                    int boundary, const void* planes, const unsigned char* mask,
                                    double threshold, long long* counts_dev, void* stream) {
    if (!mask) {
        g_last_error.clear();
        return fail(AMAP_E_INVAL, "mask must not be NULL");
    }
    return count_peaks_bc_impl(c, dt, ny, nx, nplanes, boundary, planes, mask, threshold,
                               counts_dev, stream);
}

amap_status amap_mask_shear(amap_ctx_t c, amap_dtype dt, int ny, int nx, const unsigned char* mask,
                            const void* g1, const void* g2, void* g1_out, void* g2_out,
                            void* stream) {
    g_last_error.clear();
    if (!c) return fail(AMAP_E_INVAL, "ctx must not be NULL");
    AMAP_TRY(check_dtype(dt));
    if (ny < 1 || nx < 1 || ny > 16384 || nx > 16384)
        return fail(AMAP_E_INVAL, "field sides must be in [1, 16384] (got %d x %d)", ny, nx);
    AMAP_TRY(check_ptr(mask, "mask"));
    AMAP_TRY(check_ptr(g1, "g1"));
    AMAP_TRY(check_ptr(g2, "g2"));
    AMAP_TRY(check_ptr(g1_out, "g1_out"));
    AMAP_TRY(check_ptr(g2_out, "g2_out"));
    const long long cnt = (long long)ny * nx;
    const size_t plane = (size_t)cnt * esize(dt);
    // each output is its own input or apart from every other buffer
    if ((g1_out != g1 && (overlaps(g1_out, plane, g1, plane) || overlaps(g1_out, plane, g2, plane))) ||
        (g2_out != g2 && (overlaps(g2_out, plane, g1, plane) || overlaps(g2_out, plane, g2, plane))) ||
        overlaps(g1_out, plane, g2_out, plane) || overlaps(g1_out, plane, mask, (size_t)cnt) ||
        overlaps(g2_out, plane, mask, (size_t)cnt))
        return fail(AMAP_E_INVAL, "each output must be its own input or overlap nothing");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(AMAP_E_HIP, "cannot select device %d", c->device);
    TimerScope ts(c);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (dt == AMAP_F32)
        AMAP_HIP(launch_mask_shear<float>(cnt, (const float*)g1, (const float*)g2, mask, (float*)g1_out,
                                          (float*)g2_out, s), "mask kernel");
    else
        AMAP_HIP(launch_mask_shear<double>(cnt, (const double*)g1, (const double*)g2, mask,
                                           (double*)g1_out, (double*)g2_out, s), "mask kernel");
    return AMAP_OK;
}

}  // extern "C"

// Realisations per launch of the bounded noise path: as many as fit about
// 1 GiB of workspace (P^2 spectrum, padded shears and kappa per
// realisation, plus its field-sized kappa, scratch and planes), 1 .. 32.
static int bounded_noise_batch(int ny, int nx, int P, int J, size_t esz, int n_real) {
    const size_t per = 5 * (size_t)P * P * esz + (size_t)(2 + J) * ny * nx * esz;
    size_t b = ((size_t)1 << 30) / per;
    if (b < 1) b = 1;
    if (b > 32) b = 32;
    if (b > (size_t)n_real) b = (size_t)n_real;
    return (int)b;
}
static size_t bounded_noise_bytes(int ny, int nx, int P, int J, size_t esz, int B) {
    const size_t pp = (size_t)P * P * esz * B, ff = (size_t)ny * nx * esz * B;
    return align256(2 * pp) + 3 * align256(pp) + 2 * align256(ff) + align256(ff * J) +
           2 * align256((size_t)(J - 1) * ny * nx * 8);
}

template <typename T>
static amap_status enqueue_noise_bc(const amap_ctx* c, char* w, int ny, int nx, int P, int J,
                                    int boundary, const T* g1, const T* g2, int n_real, uint64_t seed,
                                    const T* planes_signal, T* sigma, T* snr, hipStream_t s) {
    const int B = bounded_noise_batch(ny, nx, P, J, sizeof(T), n_real);
    const long long pn = (long long)P * P, fn = (long long)ny * nx;
    const size_t pp = (size_t)pn * sizeof(T) * B, ff = (size_t)fn * sizeof(T) * B;
    const long long cnt = (long long)(J - 1) * fn;
    char* q = w;
    cpx<T>* C = reinterpret_cast<cpx<T>*>(q);  q += align256(2 * pp);
    T* p1 = reinterpret_cast<T*>(q);           q += align256(pp);
    T* p2 = reinterpret_cast<T*>(q);           q += align256(pp);
    T* ke = reinterpret_cast<T*>(q);           q += align256(pp);
    T* kap = reinterpret_cast<T*>(q);          q += align256(ff);
    T* tmp = reinterpret_cast<T*>(q);          q += align256(ff);
    T* pl = reinterpret_cast<T*>(q);           q += align256(ff * J);
    double* M = reinterpret_cast<double*>(q);  q += align256((size_t)cnt * 8);
    double* M2 = reinterpret_cast<double*>(q);
    // the grids outside the field stay zero: the KS never writes its inputs
    AMAP_HIP(launch_zero2<T>(p1, p2, pn * B, s), "zero kernel");
    for (int r0 = 0; r0 < n_real; r0 += B) {
        const int nb = n_real - r0 < B ? n_real - r0 : B;
        AMAP_HIP(launch_rotate_scatter<T>(g1, g2, ny, nx, P, seed, (uint64_t)r0, nb, p1, p2, pn, s),
                 "rotation kernel");
        AMAP_TRY(enqueue_ks<T>(c, ilog2(P), nb, p1, p2, pn, C, ke, nullptr, pn, false, 0, 0, s,
                               /*pair_e=*/true));
        AMAP_HIP(launch_crop2<T>(ke, nullptr, P, ny, nx, kap, nullptr, nb, pn, fn, s), "crop kernel");
        AMAP_HIP(launch_starlet_bc<T>(ny, nx, J, boundary, kap, pl, tmp, nb, fn, (long long)J * fn, s),
                 "bounded starlet kernels");
        AMAP_HIP(launch_welford_bc<T>(pl, (long long)J * fn, nb, M, M2, cnt, r0, s), "statistics kernel");
    }
    AMAP_HIP(launch_sigma_snr_bc<T>(M2, n_real, planes_signal, sigma, snr, cnt, s), "sigma kernel");
    return AMAP_OK;
}

extern "C" {

amap_status amap_noise_maps_bc(amap_ctx_t c, amap_dtype dt, int ny, int nx, int P, int J,
                               int boundary, const void* g1, const void* g2, int n_real,
                               uint64_t seed, const void* planes_signal, void* sigma, void* snr,
                               void* stream) {
    g_last_error.clear();
    if (!c) return fail(AMAP_E_INVAL, "ctx must not be NULL");
    AMAP_TRY(check_dtype(dt));
    AMAP_TRY(check_n(P));
    if (ny < 2 || nx < 2 || ny > P || nx > P)
        return fail(AMAP_E_INVAL, "field %d x %d must have sides >= 2 and fit the %d x %d grid", ny, nx,
                    P, P);
    if (J < 2 || J > 16) return fail(AMAP_E_INVAL, "J must be in [2, 16] (got %d)", J);
    if (boundary < AMAP_BC_PERIODIC || boundary > AMAP_BC_ZERO)
        return fail(AMAP_E_INVAL, "boundary must be AMAP_BC_PERIODIC, _MIRROR or _ZERO (got %d)", boundary);
    if (n_real < 2) return fail(AMAP_E_INVAL, "n_real must be >= 2 (got %d)", n_real);
    AMAP_TRY(check_ptr(g1, "g1"));
    AMAP_TRY(check_ptr(g2, "g2"));
    AMAP_TRY(check_ptr(sigma, "sigma"));
    AMAP_TRY(check_ptr(snr, "snr", false));
    if (snr) AMAP_TRY(check_ptr(planes_signal, "planes_signal (needed for snr)"));
    const size_t f = (size_t)ny * nx * esize(dt), fd = f * (J - 1);
    if (overlaps(sigma, fd, g1, f) || overlaps(sigma, fd, g2, f) || overlaps(snr, fd, g1, f) ||
        overlaps(snr, fd, g2, f) || overlaps(sigma, fd, snr, fd) ||
        overlaps(sigma, fd, planes_signal, f * J) || overlaps(snr, fd, planes_signal, f * J))
        return fail(AMAP_E_INVAL, "outputs may not overlap inputs or each other");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(AMAP_E_HIP, "cannot select device %d", c->device);
    TimerScope ts(c);
    const int B = bounded_noise_batch(ny, nx, P, J, esize(dt), n_real);
    AMAP_TRY(c->ws.reserve(bounded_noise_bytes(ny, nx, P, J, esize(dt), B)));
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(c->ws.ptr);
    if (dt == AMAP_F32)
        return enqueue_noise_bc<float>(c, w, ny, nx, P, J, boundary, (const float*)g1, (const float*)g2,
                                       n_real, seed, (const float*)planes_signal, (float*)sigma,
                                       (float*)snr, s);
    return enqueue_noise_bc<double>(c, w, ny, nx, P, J, boundary, (const double*)g1, (const double*)g2,
                                    n_real, seed, (const double*)planes_signal, (double*)sigma,
                                    (double*)snr, s);
}

amap_status amap_starlet_reconstruct(amap_ctx_t c, amap_dtype dt, int n, int J,
                                     const void* planes, void* kappa_out, void* stream) {
    g_last_error.clear();
    if (!c) return fail(AMAP_E_INVAL, "ctx must not be NULL");
    AMAP_TRY(check_dtype(dt));
    AMAP_TRY(check_n(n));
    AMAP_TRY(check_J(n, J));
    AMAP_TRY(check_ptr(planes, "planes"));
    AMAP_TRY(check_ptr(kappa_out, "kappa_out"));
    const size_t plane = (size_t)n * n * esize(dt);
    if (overlaps(kappa_out, plane, planes, plane * J))
        return fail(AMAP_E_INVAL, "kappa_out may not overlap planes");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(AMAP_E_HIP, "cannot select device %d", c->device);
    TimerScope ts(c);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int logn = ilog2(n);
    hipError_t e = dt == AMAP_F32
        ? launch_reconstruct<float>(logn, J, (const float*)planes, (float*)kappa_out, s)
        : launch_reconstruct<double>(logn, J, (const double*)planes, (double*)kappa_out, s);
    if (e != hipSuccess) return hip_fail(e, "reconstruct kernel");
    return AMAP_OK;
}

}  // extern "C"

// Uploads the direct sum's tap tables into the context's workspace and
// launches it: the row offsets' dx ranges, the dense weights and, for the
// LDS row kernel, the weights regrouped by four dx (zero outside the disc).
template <typename T>
static amap_status enqueue_direct(amap_ctx* c, const TapTable& tab, int logn, const T* g1,
                                  const T* g2, T* out, hipStream_t s) {
    const int R = tab.R, D = 2 * R + 1;
    const int R4 = (R + 3) / 4 * 4, ng = R4 / 2 + 1;
    const bool grouped = map_direct_uses_groups(logn, R, sizeof(T));
    const size_t off_w = align256((size_t)D * sizeof(int));
    const size_t wbytes = align256((size_t)D * D * sizeof(T));
    const size_t gbytes = grouped ? align256((size_t)D * ng * 8 * sizeof(T)) : 0;
    AMAP_TRY(c->ws.reserve(off_w + 2 * wbytes + gbytes));
    char* base = static_cast<char*>(c->ws.ptr);
    std::vector<T> wc(tab.wc.begin(), tab.wc.end()), ws(tab.ws.begin(), tab.ws.end());
    std::vector<T> gt;
    if (grouped) {
        gt.assign((size_t)D * ng * 8, (T)0);
        for (int dy = -R; dy <= R; ++dy)
            for (int k = 0; k < ng; ++k)
                for (int q = 0; q < 4; ++q) {
                    const int dx = 4 * k - R4 + q;
                    if (dx < -R || dx > R) continue;
                    const size_t src = (size_t)(dy + R) * D + (dx + R);
                    const size_t dst = ((size_t)(dy + R) * ng + k) * 8;
                    gt[dst + q] = (T)tab.wc[src];
                    gt[dst + 4 + q] = (T)tab.ws[src];
                }
    }
    // The tables are staged synchronously: the workspace may still be read by
    // earlier work on this stream, so wait for it first.
    AMAP_HIP(hipStreamSynchronize(s), "stream synchronize before table upload");
    char* pc = base + off_w;
    char* ps = pc + wbytes;
    char* pg = ps + wbytes;
    AMAP_HIP(hipMemcpy(base, tab.half.data(), (size_t)D * sizeof(int), hipMemcpyHostToDevice),
             "upload tap rows");
    AMAP_HIP(hipMemcpy(pc, wc.data(), wc.size() * sizeof(T), hipMemcpyHostToDevice), "upload taps");
    AMAP_HIP(hipMemcpy(ps, ws.data(), ws.size() * sizeof(T), hipMemcpyHostToDevice), "upload taps");
    if (grouped)
        AMAP_HIP(hipMemcpy(pg, gt.data(), gt.size() * sizeof(T), hipMemcpyHostToDevice), "upload tap groups");
    AMAP_HIP(launch_map_direct<T>(logn, g1, g2, R, (const int*)base, (const T*)pc, (const T*)ps,
                                  grouped ? (const T*)pg : nullptr, out, s),
             "direct aperture-mass kernel");
    return AMAP_OK;
}

extern "C" {

amap_status amap_map_direct(amap_ctx_t c, amap_dtype dt, int n, const void* g1, const void* g2,
                            double theta_px, amap_filter filter, double fparam, double cut_px,
                            void* map_out, void* stream) {
    g_last_error.clear();
    if (!c) return fail(AMAP_E_INVAL, "ctx must not be NULL");
    AMAP_TRY(check_dtype(dt));
    AMAP_TRY(check_n(n));
    AMAP_TRY(check_ptr(g1, "g1"));
    AMAP_TRY(check_ptr(g2, "g2"));
    AMAP_TRY(check_ptr(map_out, "map_out"));
    if (!(theta_px > 0.0) || !std::isfinite(theta_px))
        return fail(AMAP_E_INVAL, "theta_px must be positive and finite");
    if (filter != AMAP_FILTER_STARLET && filter != AMAP_FILTER_S98 && filter != AMAP_FILTER_JBJ04)
        return fail(AMAP_E_INVAL, "unknown filter %d", (int)filter);
    if (filter == AMAP_FILTER_S98 && !(fparam >= 0.0))
        return fail(AMAP_E_INVAL, "S98 needs fparam = l >= 0");
    if (filter == AMAP_FILTER_JBJ04 && !(fparam > 0.0))
        return fail(AMAP_E_INVAL, "JBJ04 needs fparam = b > 0");
    const size_t bytes = (size_t)n * n * esize(dt);
    if (overlaps(map_out, bytes, g1, bytes) || overlaps(map_out, bytes, g2, bytes))
        return fail(AMAP_E_INVAL, "map_out may not overlap the inputs");
    TapTable tab;
    AMAP_TRY(build_tap_table(filter, theta_px, fparam, cut_px, n, &tab));
    DeviceGuard g(c->device);
    if (!g.ok) return fail(AMAP_E_HIP, "cannot select device %d", c->device);
    TimerScope ts(c);
    const int logn = ilog2(n);
    return dt == AMAP_F32
        ? enqueue_direct<float>(c, tab, logn, (const float*)g1, (const float*)g2, (float*)map_out,
                                static_cast<hipStream_t>(stream))
        : enqueue_direct<double>(c, tab, logn, (const double*)g1, (const double*)g2, (double*)map_out,
                                 static_cast<hipStream_t>(stream));
}

static amap_status validate_noise(amap_dtype dt, int n, int J, const void* g1, const void* g2,
                                  int n_real, const void* planes_signal, const void* sigma,
                                  const void* snr) {
    AMAP_TRY(check_dtype(dt));
    AMAP_TRY(check_n(n));
    AMAP_TRY(check_J(n, J));
    AMAP_TRY(check_ptr(g1, "g1"));
    AMAP_TRY(check_ptr(g2, "g2"));
    AMAP_TRY(check_ptr(sigma, "sigma"));
    AMAP_TRY(check_ptr(snr, "snr", false));
    AMAP_TRY(check_ptr(planes_signal, "planes_signal", snr != nullptr));
    if (n_real < 2) return fail(AMAP_E_INVAL, "n_real must be >= 2 (got %d)", n_real);
    const size_t plane = (size_t)n * n * esize(dt);
    const size_t stack = plane * (size_t)(J - 1);
    if (overlaps(sigma, stack, g1, plane) || overlaps(sigma, stack, g2, plane) ||
        overlaps(snr, stack, g1, plane) || overlaps(snr, stack, g2, plane) ||
        overlaps(sigma, stack, snr, stack) || overlaps(sigma, stack, planes_signal, plane * J) ||
        overlaps(snr, stack, planes_signal, plane * J))
        return fail(AMAP_E_INVAL, "sigma/snr may not overlap inputs or each other");
    return AMAP_OK;
}

amap_status amap_noise_maps(amap_ctx_t c, amap_dtype dt, int n, int J, const void* g1,
                            const void* g2, int n_real, uint64_t seed, const void* planes_signal,
                            void* sigma, void* snr, void* stream) {
    g_last_error.clear();
    if (!c) return fail(AMAP_E_INVAL, "ctx must not be NULL");
    AMAP_TRY(validate_noise(dt, n, J, g1, g2, n_real, planes_signal, sigma, snr));
    DeviceGuard g(c->device);
    if (!g.ok) return fail(AMAP_E_HIP, "cannot select device %d", c->device);
    TimerScope ts(c);
    AMAP_TRY(c->ws.reserve(noise_workspace_bytes(dt, n, J, n_real)));
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* ws = static_cast<char*>(c->ws.ptr);
    if (dt == AMAP_F32)
        return enqueue_noise<float>(c, ws, n, J, (const float*)g1, (const float*)g2, n_real, seed,
                                    (const float*)planes_signal, (float*)sigma, (float*)snr, s);
    return enqueue_noise<double>(c, ws, n, J, (const double*)g1, (const double*)g2, n_real, seed,
                                 (const double*)planes_signal, (double*)sigma, (double*)snr, s);
}

amap_status amap_count_peaks(amap_ctx_t c, amap_dtype dt, int n, int nplanes, const void* snr,
                             double threshold, long long* counts_dev, void* stream) {
    g_last_error.clear();
    if (!c) return fail(AMAP_E_INVAL, "ctx must not be NULL");
    AMAP_TRY(check_dtype(dt));
    AMAP_TRY(check_n(n));
    if (nplanes < 1 || nplanes > 65535) return fail(AMAP_E_INVAL, "nplanes must be in [1, 65535]");
    AMAP_TRY(check_ptr(snr, "snr"));
    if (!counts_dev) return fail(AMAP_E_INVAL, "counts_dev must not be NULL");
    if (reinterpret_cast<uintptr_t>(counts_dev) % 8 != 0)
        return fail(AMAP_E_INVAL, "counts_dev must be 8-byte aligned");
    if (std::isnan(threshold)) return fail(AMAP_E_INVAL, "threshold must not be NaN");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(AMAP_E_HIP, "cannot select device %d", c->device);
    TimerScope ts(c);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int logn = ilog2(n);
    hipError_t e = dt == AMAP_F32
        ? launch_count_peaks<float>(logn, nplanes, (const float*)snr, threshold, counts_dev, s)
        : launch_count_peaks<double>(logn, nplanes, (const double*)snr, threshold, counts_dev, s);
    if (e != hipSuccess) return hip_fail(e, "peak kernel");
    return AMAP_OK;
}

amap_status amap_peak_histogram(amap_ctx_t c, amap_dtype dt, int n, int nplanes, const void* planes,
                                int sign, double lo, double hi, int nbins, long long* hist,
                                void* stream) {
    g_last_error.clear();
    if (!c) return fail(AMAP_E_INVAL, "ctx must not be NULL");
    AMAP_TRY(check_dtype(dt));
    AMAP_TRY(check_n(n));
    if (nplanes < 1 || nplanes > 65535) return fail(AMAP_E_INVAL, "nplanes must be in [1, 65535]");
    AMAP_TRY(check_ptr(planes, "planes"));
    if (!hist || reinterpret_cast<uintptr_t>(hist) % 8 != 0)
        return fail(AMAP_E_INVAL, "hist must be a non-NULL 8-byte aligned device pointer");
    if (sign != 1 && sign != -1) return fail(AMAP_E_INVAL, "sign must be +1 or -1 (got %d)", sign);
    if (nbins < 1 || nbins > 16384) return fail(AMAP_E_INVAL, "nbins must be in [1, 16384]");
    if (!std::isfinite(lo) || !std::isfinite(hi) || !(hi > lo))
        return fail(AMAP_E_INVAL, "need finite lo < hi");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(AMAP_E_HIP, "cannot select device %d", c->device);
    TimerScope ts(c);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int logn = ilog2(n);
    const double width = (hi - lo) / (double)nbins;
    hipError_t e = dt == AMAP_F32
        ? launch_peak_hist<float>(logn, nplanes, (const float*)planes, sign, lo, width, nbins, hist, s)
        : launch_peak_hist<double>(logn, nplanes, (const double*)planes, sign, lo, width, nbins, hist, s);
    if (e != hipSuccess) return hip_fail(e, "peak histogram kernel");
    return AMAP_OK;
}

amap_status amap_plane_moments(amap_ctx_t c, amap_dtype dt, int n, int nplanes, const void* planes,
                               double* out, void* stream) {
    g_last_error.clear();
    if (!c) return fail(AMAP_E_INVAL, "ctx must not be NULL");
    AMAP_TRY(check_dtype(dt));
    AMAP_TRY(check_n(n));
    if (nplanes < 1 || nplanes > 65535) return fail(AMAP_E_INVAL, "nplanes must be in [1, 65535]");
    AMAP_TRY(check_ptr(planes, "planes"));
    if (!out || reinterpret_cast<uintptr_t>(out) % 8 != 0)
        return fail(AMAP_E_INVAL, "out must be a non-NULL 8-byte aligned device pointer");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(AMAP_E_HIP, "cannot select device %d", c->device);
    TimerScope ts(c);
    const int logn = ilog2(n);
    AMAP_TRY(c->ws.reserve((size_t)3 * nplanes * moment_blocks(logn) * sizeof(double)));
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* part = static_cast<double*>(c->ws.ptr);
    hipError_t e = dt == AMAP_F32
        ? launch_plane_moments<float>(logn, nplanes, (const float*)planes, part, out, s)
        : launch_plane_moments<double>(logn, nplanes, (const double*)planes, part, out, s);
    if (e != hipSuccess) return hip_fail(e, "moment kernels");
    return AMAP_OK;
}

amap_status amap_phase_uniforms(amap_ctx_t c, int n, uint64_t seed, uint64_t r, uint32_t* out_u32,
                                void* stream) {
    g_last_error.clear();
    if (!c) return fail(AMAP_E_INVAL, "ctx must not be NULL");
    AMAP_TRY(check_n(n));
    AMAP_TRY(check_ptr(out_u32, "out_u32"));
    DeviceGuard g(c->device);
    if (!g.ok) return fail(AMAP_E_HIP, "cannot select device %d", c->device);
    TimerScope ts(c);
    AMAP_HIP(launch_phase_u32(ilog2(n), seed, r, out_u32, static_cast<hipStream_t>(stream)),
             "phase kernel");
    return AMAP_OK;
}

static amap_status validate_job(amap_dtype dt, const amap_job& j) {
    AMAP_TRY(check_dtype(dt));
    AMAP_TRY(check_n(j.n));
    AMAP_TRY(check_J(j.n, j.J));
    AMAP_TRY(check_ptr(j.g1, "g1"));
    AMAP_TRY(check_ptr(j.g2, "g2"));
    AMAP_TRY(check_ptr(j.planes, "planes"));
    AMAP_TRY(check_ptr(j.kappa_e, "kappa_e", false));
    const size_t plane = (size_t)j.n * j.n * esize(dt);
    if (overlaps(j.planes, plane * j.J, j.g1, plane) || overlaps(j.planes, plane * j.J, j.g2, plane) ||
        overlaps(j.kappa_e, plane, j.planes, plane * j.J) || overlaps(j.kappa_e, plane, j.g1, plane) ||
        overlaps(j.kappa_e, plane, j.g2, plane))
        return fail(AMAP_E_INVAL, "outputs may not overlap inputs or each other");
    if (j.n_real == 0) return AMAP_OK;
    AMAP_TRY(check_ptr(j.snr, "snr"));
    AMAP_TRY(validate_noise(dt, j.n, j.J, j.g1, j.g2, j.n_real, j.planes, j.sigma, j.snr));
    if (!j.peaks || reinterpret_cast<uintptr_t>(j.peaks) % 8 != 0)
        return fail(AMAP_E_INVAL, "peaks must be a non-NULL 8-byte aligned device pointer");
    if (std::isnan(j.threshold)) return fail(AMAP_E_INVAL, "threshold must not be NaN");
    return AMAP_OK;
}

// Workspace of one job: [signal spectrum | signal kappa | starlet scratch | noise].
static size_t job_workspace_bytes(amap_dtype dt, const amap_job& j) {
    const size_t plane = (size_t)j.n * j.n * esize(dt);
    size_t b = align256(2 * plane) + align256(plane) + align256(2 * plane);
    if (j.n_real >= 2) b += noise_workspace_bytes(dt, j.n, j.J, j.n_real);
    return b;
}

}  // extern "C"

template <typename T>
static amap_status enqueue_job(const amap_ctx* c, char* w, const amap_job& j, hipStream_t s) {
    const size_t plane = (size_t)j.n * j.n * sizeof(T);
    const int logn = ilog2(j.n);
    const long long n2 = (long long)j.n * j.n;
    cpx<T>* C = reinterpret_cast<cpx<T>*>(w);
    T* kap = j.kappa_e ? (T*)j.kappa_e : reinterpret_cast<T*>(w + align256(2 * plane));
    T* tmp = reinterpret_cast<T*>(w + align256(2 * plane) + align256(plane));
    char* nws = w + align256(2 * plane) + align256(plane) + align256(2 * plane);
    AMAP_TRY(enqueue_ks<T>(c, logn, 1, (const T*)j.g1, (const T*)j.g2, 0, C, kap, nullptr, n2,
                           false, 0, 0, s));
    AMAP_TRY(enqueue_starlet<T>(c, logn, j.J, 1, kap, n2, (T*)j.planes, (long long)j.J * n2, tmp, s));
    if (j.n_real < 2) return AMAP_OK;
    AMAP_TRY(enqueue_noise<T>(c, nws, j.n, j.J, (const T*)j.g1, (const T*)j.g2, j.n_real, j.seed,
                              (const T*)j.planes, (T*)j.sigma, (T*)j.snr, s));
    AMAP_HIP(launch_count_peaks<T>(logn, j.J - 1, (const T*)j.snr, j.threshold, j.peaks, s),
             "peak kernel");
    return AMAP_OK;
}

extern "C" {

amap_status amap_run_path(amap_ctx_t c, amap_dtype dt, int n, int J, const void* g1,
                          const void* g2, int n_real, uint64_t seed, double threshold,
                          void* kappa_e, void* kappa_b, void* planes, void* sigma, void* snr,
                          long long* peaks, void* stream) {
    g_last_error.clear();
    if (!c) return fail(AMAP_E_INVAL, "ctx must not be NULL");
    amap_job j;
    j.n = n; j.J = J; j.n_real = n_real; j.seed = seed; j.threshold = threshold;
    j.g1 = g1; j.g2 = g2; j.kappa_e = kappa_e; j.planes = planes; j.sigma = sigma;
    j.snr = snr; j.peaks = peaks;
    if (n_real < 2) return fail(AMAP_E_INVAL, "n_real must be >= 2 (got %d)", n_real);
    AMAP_TRY(validate_job(dt, j));
    AMAP_TRY(check_ptr(kappa_b, "kappa_b", false));
    const size_t plane = (size_t)n * n * esize(dt);
    if (overlaps(kappa_b, plane, planes, plane * J) || overlaps(kappa_b, plane, g1, plane) ||
        overlaps(kappa_b, plane, g2, plane) || overlaps(kappa_b, plane, kappa_e, plane))
        return fail(AMAP_E_INVAL, "kappa_b may not overlap inputs or other outputs");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(AMAP_E_HIP, "cannot select device %d", c->device);
    TimerScope ts(c);
    AMAP_TRY(c->ws.reserve(job_workspace_bytes(dt, j)));
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(c->ws.ptr);
    if (kappa_b) {
        // kappa_B is an extra output of the signal's KS pass only
        AMAP_TRY(dt == AMAP_F32
                 ? enqueue_ks<float>(c, ilog2(n), 1, (const float*)g1, (const float*)g2, 0,
                                     (cpx<float>*)w, (float*)(w + align256(2 * plane)),
                                     (float*)kappa_b, (long long)n * n, false, 0, 0, s)
                 : enqueue_ks<double>(c, ilog2(n), 1, (const double*)g1, (const double*)g2, 0,
                                      (cpx<double>*)w, (double*)(w + align256(2 * plane)),
                                      (double*)kappa_b, (long long)n * n, false, 0, 0, s));
    }
    return dt == AMAP_F32 ? enqueue_job<float>(c, w, j, s) : enqueue_job<double>(c, w, j, s);
}

size_t amap_job_footprint_bytes(amap_dtype dt, int n, int J, int n_real) {
    if (check_dtype(dt) != AMAP_OK || check_n(n) != AMAP_OK || check_J(n, J) != AMAP_OK) return 0;
    amap_job j;
    std::memset(&j, 0, sizeof j);
    j.n = n; j.J = J; j.n_real = n_real >= 2 ? n_real : 0;
    return job_workspace_bytes(dt, j);
}

int amap_noise_batch(int n, int n_real) {
    if (check_n(n) != AMAP_OK || n_real < 2) return 0;
    return noise_batch(n, n_real);
}

}  // extern "C"

// A batch plan.  Jobs without noise realisations whose size has an LDS tile
// for every starlet stage are grouped by (n, J) into chunks; one chunk runs
// as one launch per kernel, the maps addressed through device tables of
// per-map pointers.  Other jobs (noise, untiled sizes) run one after another.
struct PlanChunk {
    int n, J, count;
    size_t tab_off;              // byte offset of the chunk's tables in amap_plan::tabs
    char* base[4];               // g1, g2, kappa, planes of the chunk's first map
};

// Lanes of a plan: lane 0 runs the grouped chunks, lanes 1.. the jobs that
// run alone (those with noise, or shapes without grouped kernels), each lane
// in order on its own workspace region.  In a captured graph the lanes are
// branches forked from and joined back into the caller's stream, so jobs of
// different lanes overlap on the device.
constexpr int kPlanLanes = 4;                  // lanes for jobs that run alone
constexpr size_t kPlanLaneBytes = 16ull << 30;  // more lanes only within this much workspace

struct amap_plan {
    amap_ctx* ctx = nullptr;
    amap_dtype dt = AMAP_F32;
    std::vector<amap_job> jobs;
    std::vector<PlanChunk> chunks;
    std::vector<int> singles;    // indices of jobs run one at a time
    std::vector<int> lane_of;    // lane (1..) of each entry of singles
    std::vector<size_t> lane_off;  // workspace offset of each lane (lane 0: chunks)
    int lanes = 1;
    void* tabs = nullptr;        // device: per chunk [g1 | g2 | kappa | planes] x count offsets
    Workspace ws;
    hipStream_t graph_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<hipStream_t> branch;  // lanes 1.. while capturing (default priority)
    std::vector<hipEvent_t> ev;       // fork event, then one join event per lane
    void drop_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        graph_stream = nullptr;
    }
    void drop_streams() {
        for (hipStream_t b : branch) (void)hipStreamDestroy(b);
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        branch.clear();
        ev.clear();
    }
};

// Device bytes a chunk of `count` maps needs: spectra, kappa slots and the two
// c buffers of the starlet stages.
static size_t chunk_workspace_bytes(amap_dtype dt, int n, int count) {
    const size_t plane = (size_t)n * n * esize(dt);
    return align256(2 * plane * count) + 3 * align256(plane * count);
}

constexpr size_t kChunkBytes = 2ull << 30;  // workspace of one grouped chunk, at most

template <typename T>
static amap_status enqueue_chunk(const amap_plan* p, const PlanChunk& ch, hipStream_t s) {
    const size_t plane = (size_t)ch.n * ch.n * sizeof(T);
    const int logn = ilog2(ch.n);
    const long long n2 = (long long)ch.n * ch.n;
    char* w = static_cast<char*>(p->ws.ptr);
    cpx<T>* C = reinterpret_cast<cpx<T>*>(w);
    T* cb0 = reinterpret_cast<T*>(w + align256(2 * plane * ch.count) + align256(plane * ch.count));
    T* cb1 = reinterpret_cast<T*>(reinterpret_cast<char*>(cb0) + align256(plane * ch.count));
    // tables: [g1 | g2 | kappa | planes] x count element offsets from the
    // chunk's base pointers
    const long long* off = reinterpret_cast<const long long*>(static_cast<char*>(p->tabs) + ch.tab_off);
    KsArgs<T> k;
    k.logn = logn; k.batch = ch.count; k.g1 = (const T*)ch.base[0]; k.g2 = (const T*)ch.base[1];
    k.g_stride = 0; k.C = C; k.kE = (T*)ch.base[2]; k.kB = nullptr; k.out_stride = n2;
    k.rotate = false; k.seed = 0; k.r0 = 0; k.tw = twiddles<T>(p->ctx); k.stream = s;
    k.g1_off = off; k.g2_off = off + ch.count; k.kE_off = off + 2 * ch.count;
    AMAP_HIP(launch_ks<T>(k), "KS kernels (grouped)");
    StarletArgs<T> a;
    a.logn = logn; a.J = ch.J; a.batch = ch.count; a.done = 0; a.kappa = (const T*)ch.base[2];
    a.in_stride = n2; a.planes = (T*)ch.base[3]; a.planes_stride = 0; a.cbuf0 = cb0; a.cbuf1 = cb1;
    a.tmp = nullptr; a.wbuf = nullptr; a.M = nullptr; a.M2 = nullptr; a.part = nullptr; a.stream = s;
    a.kappa_off = off + 2 * ch.count;
    a.planes_off = off + 3 * ch.count;
    a.plan = tuned_plan<T>(p->ctx, a);
    AMAP_HIP(launch_starlet<T>(a), "starlet kernels (grouped)");
    return AMAP_OK;
}

// Every lane's work in lane order on its stream: lanes[l] (lanes[0] = s).
static amap_status enqueue_lanes(amap_plan* p, const hipStream_t* lanes) {
    for (const PlanChunk& ch : p->chunks)
        AMAP_TRY(p->dt == AMAP_F32 ? enqueue_chunk<float>(p, ch, lanes[0])
                                   : enqueue_chunk<double>(p, ch, lanes[0]));
    char* w = static_cast<char*>(p->ws.ptr);
    for (size_t k = 0; k < p->singles.size(); ++k) {
        const amap_job& j = p->jobs[p->singles[k]];
        const int l = p->lane_of[k];
        char* wl = w + p->lane_off[l];
        AMAP_TRY(p->dt == AMAP_F32 ? enqueue_job<float>(p->ctx, wl, j, lanes[l])
                                   : enqueue_job<double>(p->ctx, wl, j, lanes[l]));
    }
    return AMAP_OK;
}

// All of the plan on stream s, lane after lane (the lanes' workspace
// regions are disjoint, so one stream gives the same results).
static amap_status enqueue_plan(amap_plan* p, hipStream_t s) {
    std::vector<hipStream_t> lanes(p->lanes, s);
    return enqueue_lanes(p, lanes.data());
}

// The plan as branches of the stream being captured: fork every lane from
// s, join them all back into s.
static amap_status enqueue_plan_forked(amap_plan* p, hipStream_t s) {
    if (p->lanes == 1) return enqueue_plan(p, s);
    if (p->branch.empty()) {
        p->branch.assign(p->lanes - 1, nullptr);
        p->ev.assign(p->lanes, nullptr);
        for (hipStream_t& b : p->branch)
            AMAP_HIP(hipStreamCreateWithFlags(&b, hipStreamNonBlocking), "lane stream");
        for (hipEvent_t& e : p->ev) AMAP_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming), "lane event");
    }
    std::vector<hipStream_t> lanes(p->lanes, s);
    AMAP_HIP(hipEventRecord(p->ev[0], s), "fork");
    for (int l = 1; l < p->lanes; ++l) {
        lanes[l] = p->branch[l - 1];
        AMAP_HIP(hipStreamWaitEvent(lanes[l], p->ev[0], 0), "fork wait");
    }
    AMAP_TRY(enqueue_lanes(p, lanes.data()));
    for (int l = 1; l < p->lanes; ++l) {
        AMAP_HIP(hipEventRecord(p->ev[l], lanes[l]), "join");
        AMAP_HIP(hipStreamWaitEvent(s, p->ev[l], 0), "join wait");
    }
    return AMAP_OK;
}

extern "C" {

amap_status amap_batch_plan(amap_ctx_t c, amap_dtype dt, const amap_job* jobs, int njobs,
                            amap_plan_t* out) {
    g_last_error.clear();
    if (!c) return fail(AMAP_E_INVAL, "ctx must not be NULL");
    if (!out) return fail(AMAP_E_INVAL, "out must not be NULL");
    *out = nullptr;
    if (njobs < 1 || !jobs) return fail(AMAP_E_INVAL, "need at least one job");
    for (int i = 0; i < njobs; ++i) {
        amap_status st = validate_job(dt, jobs[i]);
        if (st != AMAP_OK) {
            std::string m = g_last_error;
            return fail(st, "job %d: %s", i, m.c_str());
        }
        if (jobs[i].n_real == 1 || jobs[i].n_real < 0)
            return fail(AMAP_E_INVAL, "job %d: n_real must be 0 or >= 2", i);
    }
    DeviceGuard g(c->device);
    if (!g.ok) return fail(AMAP_E_HIP, "cannot select device %d", c->device);
    TimerScope ts(c);
    amap_plan* p = new (std::nothrow) amap_plan;
    if (!p) return fail(AMAP_E_NOMEM, "out of host memory");
    p->ctx = c;
    p->dt = dt;
    p->jobs.assign(jobs, jobs + njobs);
    // group: (n, J) -> job indices, in job order
    std::map<std::pair<int, int>, std::vector<int>> groups;
    for (int i = 0; i < njobs; ++i) {
        const amap_job& j = jobs[i];
        const bool tiled = dt == AMAP_F32 ? starlet_all_tiled<float>(j.n, j.J)
                                          : starlet_all_tiled<double>(j.n, j.J);
        if (j.n_real == 0 && tiled) groups[{j.n, j.J}].push_back(i);
        else p->singles.push_back(i);
    }
    size_t need = 0, tab_bytes = 0;
    for (auto& kv : groups) {
        const int n = kv.first.first, J = kv.first.second;
        const size_t per = chunk_workspace_bytes(dt, n, 1);
        const int cap = (int)std::max<size_t>(1, kChunkBytes / per);
        const std::vector<int>& idx = kv.second;
        for (size_t k = 0; k < idx.size(); k += cap) {
            const int cnt = (int)std::min<size_t>(cap, idx.size() - k);
            p->chunks.push_back(PlanChunk{n, J, cnt, tab_bytes, {nullptr, nullptr, nullptr, nullptr}});
            tab_bytes += align256(4 * sizeof(long long) * cnt);
            need = std::max(need, chunk_workspace_bytes(dt, n, cnt));
        }
    }
    // lanes for the jobs that run alone: each job to the lane with the
    // least work so far (work ~ pixels x (1 + realisations)), as many lanes
    // as the workspace bound allows (one at least)
    size_t single_max = 0;
    for (int i : p->singles) single_max = std::max(single_max, job_workspace_bytes(dt, jobs[i]));
    int nl = std::min<int>(kPlanLanes, (int)p->singles.size());
    while (nl > 1 && need + (size_t)nl * single_max > kPlanLaneBytes) --nl;
    p->lanes = 1 + std::max(nl, p->singles.empty() ? 0 : 1);
    std::vector<double> load(p->lanes, 0.0);
    std::vector<size_t> lane_need(p->lanes, 0);
    lane_need[0] = need;
    for (int i : p->singles) {
        int best = 1;
        for (int l = 2; l < p->lanes; ++l)
            if (load[l] < load[best]) best = l;
        load[best] += (double)jobs[i].n * jobs[i].n * (1.0 + jobs[i].n_real);
        lane_need[best] = std::max(lane_need[best], job_workspace_bytes(dt, jobs[i]));
        p->lane_of.push_back(best);
    }
    p->lane_off.assign(p->lanes, 0);
    for (int l = 1; l < p->lanes; ++l) p->lane_off[l] = p->lane_off[l - 1] + align256(lane_need[l - 1]);
    need = p->lane_off[p->lanes - 1] + lane_need[p->lanes - 1];
    amap_status st = p->ws.reserve(need);
    if (st == AMAP_OK && tab_bytes) {
        std::vector<long long> host(tab_bytes / sizeof(long long), 0);
        char* ws = static_cast<char*>(p->ws.ptr);
        const size_t es = esize(dt);
        size_t ci = 0;
        for (auto& kv : groups) {
            const int n = kv.first.first;
            const size_t plane = (size_t)n * n * es;
            const std::vector<int>& idx = kv.second;
            for (size_t k = 0; k < idx.size();) {
                PlanChunk& ch = p->chunks[ci++];
                long long* t = host.data() + ch.tab_off / sizeof(long long);
                char* kslot = ws + align256(2 * plane * ch.count);
                for (int m = 0; m < ch.count; ++m, ++k) {
                    const amap_job& j = jobs[idx[k]];
                    char* ptr[4] = {(char*)j.g1, (char*)j.g2,
                                    j.kappa_e ? (char*)j.kappa_e : kslot + plane * m, (char*)j.planes};
                    for (int q = 0; q < 4; ++q) {
                        if (m == 0) ch.base[q] = ptr[q];
                        // element offset from the chunk's base (buffers are 256-byte aligned)
                        t[q * ch.count + m] = (long long)((intptr_t)ptr[q] - (intptr_t)ch.base[q]) / (long long)es;
                    }
                }
            }
        }
        if (hipMalloc(&p->tabs, tab_bytes) != hipSuccess) {
            st = fail(AMAP_E_NOMEM, "cannot allocate %zu bytes of map tables", tab_bytes);
        } else if (hipMemcpy(p->tabs, host.data(), tab_bytes, hipMemcpyHostToDevice) != hipSuccess) {
            st = fail(AMAP_E_HIP, "cannot upload map tables");
        }
    }
    if (st == AMAP_OK && c->autotune == 1) {
        // one direct run on the null stream tunes (and caches) the starlet
        // schedule of every group and job shape before any graph capture
        st = enqueue_plan(p, nullptr);
        if (st == AMAP_OK && hipDeviceSynchronize() != hipSuccess)
            st = fail(AMAP_E_HIP, "plan warm-up run failed");
    }
    if (st != AMAP_OK) {
        if (p->tabs) (void)hipFree(p->tabs);
        p->ws.release();
        delete p;
        return st;
    }
    *out = p;
    return AMAP_OK;
}

amap_status amap_batch_run(amap_plan_t p, void* stream) {
    g_last_error.clear();
    if (!p) return fail(AMAP_E_INVAL, "plan must not be NULL");
    DeviceGuard g(p->ctx->device);
    if (!g.ok) return fail(AMAP_E_HIP, "cannot select device %d", p->ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!s) {  // the null stream cannot be captured: launch directly (timed if enabled)
        TimerScope ts(p->ctx);
        return enqueue_plan(p, s);
    }
    if (!p->exec || p->graph_stream != s) {
        p->drop_graph();
        AMAP_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "begin capture");
        amap_status st = enqueue_plan_forked(p, s);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(s, &graph);
        if (st != AMAP_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess) return hip_fail(e, "end capture");
        p->graph = graph;
        e = hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            p->drop_graph();
            return hip_fail(e, "graph instantiate");
        }
        p->graph_stream = s;
    }
    AMAP_HIP(hipGraphLaunch(p->exec, s), "graph launch");
    return AMAP_OK;
}

amap_status amap_plan_destroy(amap_plan_t p) {
    g_last_error.clear();
    if (!p) return AMAP_OK;
    DeviceGuard g(p->ctx->device);
    (void)hipDeviceSynchronize();
    p->drop_graph();
    p->drop_streams();
    if (p->tabs) (void)hipFree(p->tabs);
    p->ws.release();
    delete p;
    return AMAP_OK;
}

}  // extern "C"

// ---- serving ------------------------------------------------------------------------
struct amap_server {
    struct Slot {
        hipStream_t stream = nullptr;
        hipEvent_t done = nullptr;
        long long ticket = -1;    // job on the device, or -1
        size_t footprint = 0;
        size_t offset = 0;        // of its workspace in the arena
    };
    struct Pending {
        long long ticket;
        amap_job job;
        size_t footprint;
        hipEvent_t ready;         // recorded on the submitting stream at submit
    };
    amap_ctx* ctx = nullptr;
    amap_dtype dt = AMAP_F32;
    size_t budget = 0, in_use = 0;
    int max_queued = 0;
    long long next_ticket = 0;
    std::vector<Slot> slots;
    std::vector<Pending> queue;               // FIFO (front = oldest)
    std::map<long long, int> state;           // 0 queued, 1 on the device, 2 done
    std::vector<long long> finished;          // done, not yet reported by amap_server_completed
    char* arena = nullptr;                    // mem_budget bytes of device memory, allocated once
    std::map<size_t, size_t> holes;           // free ranges of the arena: offset -> length
    std::vector<hipEvent_t> events;           // reusable submit events

    hipEvent_t get_event() {
        hipEvent_t e = nullptr;
        if (!events.empty()) {
            e = events.back();
            events.pop_back();
        } else if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            e = nullptr;
        }
        return e;
    }

    // First fit of `bytes` (a multiple of 256) in the arena; false if no hole fits.
    bool take(size_t bytes, size_t* off) {
        for (auto it = holes.begin(); it != holes.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes;
            holes.erase(it);
            if (rest) holes[*off + bytes] = rest;
            return true;
        }
        return false;
    }
    void give(size_t off, size_t bytes) {
        auto it = holes.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != holes.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            holes.erase(nx);
        }
        if (it != holes.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                holes.erase(it);
            }
        }
    }
};

namespace {

// Enqueue one admitted job on its slot, its workspace at `off` in the arena.
amap_status launch_on_slot(amap_server* v, amap_server::Slot& sl, const amap_server::Pending& p,
                           size_t off) {
    TimerScope ts(v->ctx);
    char* w = v->arena + off;
    // the job runs after the work its submitter enqueued before submitting
    AMAP_HIP(hipStreamWaitEvent(sl.stream, p.ready, 0), "wait for the submitting stream");
    AMAP_TRY(v->dt == AMAP_F32 ? enqueue_job<float>(v->ctx, w, p.job, sl.stream)
                               : enqueue_job<double>(v->ctx, w, p.job, sl.stream));
    AMAP_HIP(hipEventRecord(sl.done, sl.stream), "done event");
    sl.ticket = p.ticket;
    sl.footprint = p.footprint;
    sl.offset = off;
    v->in_use += p.footprint;
    v->state[p.ticket] = 1;
    return AMAP_OK;
}

// Retire finished slots, then admit queued jobs in order while a slot is
// free and the budget allows (a job that does not fit blocks those behind it,
// so large jobs are not starved).
amap_status pump(amap_server* v) {
    for (amap_server::Slot& sl : v->slots) {
        if (sl.ticket < 0) continue;
        const hipError_t e = hipEventQuery(sl.done);
        if (e == hipErrorNotReady) continue;
        if (e != hipSuccess) return fail(AMAP_E_HIP, "job %lld: %s", sl.ticket, hipGetErrorString(e));
        v->state[sl.ticket] = 2;
        v->finished.push_back(sl.ticket);
        v->in_use -= sl.footprint;
        v->give(sl.offset, sl.footprint);
        sl.ticket = -1;
        sl.footprint = 0;
    }
    while (!v->queue.empty()) {
        const amap_server::Pending& p = v->queue.front();
        amap_server::Slot* free_slot = nullptr;
        for (amap_server::Slot& sl : v->slots)
            if (sl.ticket < 0) { free_slot = &sl; break; }
        if (!free_slot) break;
        size_t off = 0;
        if (!v->take(p.footprint, &off)) break;  // wait for memory
        const amap_status st = launch_on_slot(v, *free_slot, p, off);
        if (st != AMAP_OK) {
            v->give(off, p.footprint);
            return st;
        }
        // the slot's wait has taken the event's state; it can be recorded again
        v->events.push_back(p.ready);
        v->queue.erase(v->queue.begin());
    }
    return AMAP_OK;
}

}  // namespace

extern "C" {

amap_status amap_server_create(amap_ctx_t c, amap_dtype dt, size_t mem_budget, int max_inflight,
                               int max_queued, amap_server_t* out) {
    g_last_error.clear();
    if (!c) return fail(AMAP_E_INVAL, "ctx must not be NULL");
    if (!out) return fail(AMAP_E_INVAL, "out must not be NULL");
    *out = nullptr;
    AMAP_TRY(check_dtype(dt));
    if (max_inflight < 1 || max_inflight > 64)
        return fail(AMAP_E_INVAL, "max_inflight must be in [1, 64] (got %d)", max_inflight);
    if (max_queued < 1) return fail(AMAP_E_INVAL, "max_queued must be >= 1 (got %d)", max_queued);
    if (mem_budget == 0) return fail(AMAP_E_INVAL, "mem_budget must be > 0");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(AMAP_E_HIP, "cannot select device %d", c->device);
    amap_server* v = new (std::nothrow) amap_server;
    if (!v) return fail(AMAP_E_NOMEM, "out of host memory");
    v->ctx = c;
    v->dt = dt;
    v->max_queued = max_queued;
    v->slots.resize(max_inflight);
    // one arena for all admitted workspaces: no allocation while serving
    v->budget = mem_budget / 256 * 256;
    if (v->budget == 0 || hipMalloc(&v->arena, v->budget) != hipSuccess) {
        (void)hipGetLastError();
        delete v;
        return fail(AMAP_E_NOMEM, "cannot allocate the %zu-byte server arena", mem_budget);
    }
    v->holes[0] = v->budget;
    for (amap_server::Slot& sl : v->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
            for (amap_server::Slot& t : v->slots) {
                if (t.done) (void)hipEventDestroy(t.done);
                if (t.stream) (void)hipStreamDestroy(t.stream);
            }
            (void)hipFree(v->arena);
            delete v;
            return fail(AMAP_E_HIP, "cannot create server streams");
        }
    }
    *out = v;
    return AMAP_OK;
}

amap_status amap_server_submit(amap_server_t v, const amap_job* job, void* stream,
                               long long* ticket) {
    g_last_error.clear();
    if (!v) return fail(AMAP_E_INVAL, "server must not be NULL");
    if (!job || !ticket) return fail(AMAP_E_INVAL, "job and ticket must not be NULL");
    AMAP_TRY(validate_job(v->dt, *job));
    if (job->n_real == 1 || job->n_real < 0)
        return fail(AMAP_E_INVAL, "n_real must be 0 or >= 2 (got %d)", job->n_real);
    const size_t fp = align256(job_workspace_bytes(v->dt, *job));
    if (fp > v->budget)
        return fail(AMAP_E_NOMEM, "job needs %zu bytes of workspace, over the budget of %zu", fp,
                    v->budget);
    DeviceGuard g(v->ctx->device);
    if (!g.ok) return fail(AMAP_E_HIP, "cannot select device %d", v->ctx->device);
    AMAP_TRY(pump(v));
    if ((int)v->queue.size() >= v->max_queued) return fail(AMAP_E_BUSY, "queue full");
    hipEvent_t ev = v->get_event();
    if (!ev) return fail(AMAP_E_HIP, "cannot create a submit event");
    const hipError_t er = hipEventRecord(ev, static_cast<hipStream_t>(stream));
    if (er != hipSuccess) {
        v->events.push_back(ev);
        return hip_fail(er, "record the submit event");
    }
    const long long t = v->next_ticket++;
    v->queue.push_back(amap_server::Pending{t, *job, fp, ev});
    v->state[t] = 0;
    *ticket = t;
    return pump(v);
}

amap_status amap_server_poll(amap_server_t v, long long ticket, int* done) {
    g_last_error.clear();
    if (!v || !done) return fail(AMAP_E_INVAL, "server and done must not be NULL");
    auto it = v->state.find(ticket);
    if (it == v->state.end()) return fail(AMAP_E_INVAL, "unknown ticket %lld", ticket);
    DeviceGuard g(v->ctx->device);
    if (!g.ok) return fail(AMAP_E_HIP, "cannot select device %d", v->ctx->device);
    AMAP_TRY(pump(v));
    *done = v->state[ticket] == 2;
    return AMAP_OK;
}

amap_status amap_server_completed(amap_server_t v, long long* out, int cap, int* count) {
    g_last_error.clear();
    if (!v || !count || (cap > 0 && !out)) return fail(AMAP_E_INVAL, "bad arguments");
    DeviceGuard g(v->ctx->device);
    if (!g.ok) return fail(AMAP_E_HIP, "cannot select device %d", v->ctx->device);
    AMAP_TRY(pump(v));
    std::sort(v->finished.begin(), v->finished.end());
    const int k = std::min<int>(cap, (int)v->finished.size());
    for (int i = 0; i < k; ++i) out[i] = v->finished[i];
    v->finished.erase(v->finished.begin(), v->finished.begin() + k);
    *count = k;
    return AMAP_OK;
}

amap_status amap_server_wait(amap_server_t v, long long ticket) {
    g_last_error.clear();
    if (!v) return fail(AMAP_E_INVAL, "server must not be NULL");
    if (v->state.find(ticket) == v->state.end()) return fail(AMAP_E_INVAL, "unknown ticket %lld", ticket);
    DeviceGuard g(v->ctx->device);
    if (!g.ok) return fail(AMAP_E_HIP, "cannot select device %d", v->ctx->device);
    for (;;) {
        AMAP_TRY(pump(v));
        if (v->state[ticket] == 2) return AMAP_OK;
        // block on the oldest job on the device, then retire and admit again
        amap_server::Slot* busy = nullptr;
        for (amap_server::Slot& sl : v->slots)
            if (sl.ticket >= 0 && (!busy || sl.ticket < busy->ticket)) busy = &sl;
        if (!busy) return fail(AMAP_E_HIP, "ticket %lld cannot be admitted", ticket);
        const hipError_t e = hipEventSynchronize(busy->done);
        if (e != hipSuccess)
            return fail(AMAP_E_HIP, "wait for job %lld: %s", busy->ticket, hipGetErrorString(e));
    }
}

amap_status amap_server_stats(amap_server_t v, int* queued, int* inflight, size_t* mem_in_use) {
    g_last_error.clear();
    if (!v) return fail(AMAP_E_INVAL, "server must not be NULL");
    int n = 0;
    for (const amap_server::Slot& sl : v->slots) n += sl.ticket >= 0;
    if (queued) *queued = (int)v->queue.size();
    if (inflight) *inflight = n;
    if (mem_in_use) *mem_in_use = v->in_use;
    return AMAP_OK;
}

amap_status amap_server_destroy(amap_server_t v) {
    g_last_error.clear();
    if (!v) return AMAP_OK;
    DeviceGuard g(v->ctx->device);
    amap_status st = AMAP_OK;
    // run what is still queued, then drain
    while (st == AMAP_OK && !v->queue.empty()) {
        st = pump(v);
        for (amap_server::Slot& sl : v->slots)
            if (sl.ticket >= 0) (void)hipEventSynchronize(sl.done);
    }
    for (amap_server::Slot& sl : v->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    for (const amap_server::Pending& p : v->queue)  // left behind only after an error
        if (p.ready) (void)hipEventDestroy(p.ready);
    for (hipEvent_t e : v->events) (void)hipEventDestroy(e);
    if (v->arena) (void)hipFree(v->arena);
    delete v;
    return st;
}

}  // extern "C"

