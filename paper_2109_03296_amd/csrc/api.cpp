// Status strings, per-thread error text, version, shared argument checks.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "kbm_internal.h"

namespace kbm {

static thread_local std::string g_last_error;

void set_error(const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

void clear_error() { g_last_error.clear(); }

kbm_status check_stack(const kbm_stack *s, const char *what) {
    KBM_REQUIRE(s != nullptr, KBM_ERR_INVALID_ARG, "%s: stack is NULL", what);
    KBM_REQUIRE(s->width >= 1 && s->height >= 1, KBM_ERR_INVALID_ARG,
                "%s: image size %d x %d must be positive", what, s->width,
                s->height);
    KBM_REQUIRE(s->width <= (1 << 20) && s->height <= (1 << 20),
                KBM_ERR_UNSUPPORTED, "%s: image side exceeds 2^20", what);
    KBM_REQUIRE((int64_t)s->width * s->height < (int64_t)1 << 31,
                KBM_ERR_UNSUPPORTED, "%s: W*H = %lld exceeds 2^31", what,
                (long long)s->width * s->height);
    KBM_REQUIRE(s->num_epochs >= 1 && s->num_epochs <= KBM_MAX_EPOCHS,
                KBM_ERR_INVALID_ARG, "%s: num_epochs %d not in [1, %d]", what,
                s->num_epochs, KBM_MAX_EPOCHS);
    KBM_REQUIRE(s->times != nullptr, KBM_ERR_INVALID_ARG, "%s: times is NULL",
                what);
    for (int i = 0; i < s->num_epochs; ++i)
        KBM_REQUIRE(std::isfinite(s->times[i]), KBM_ERR_INVALID_ARG,
                    "%s: times[%d] is not finite", what, i);
    return KBM_OK;
}

kbm_status check_sigmag_params(double q_lo, double q_hi, double coeff,
                               double n_sigma) {
    KBM_REQUIRE(std::isfinite(q_lo) && std::isfinite(q_hi) && q_lo >= 0.0 &&
                    q_lo < q_hi && q_hi <= 1.0,
                KBM_ERR_INVALID_ARG, "quantiles need 0 <= q_lo < q_hi <= 1 (got %g, %g)",
                q_lo, q_hi);
    KBM_REQUIRE(std::isfinite(coeff) && coeff >= 0.0, KBM_ERR_INVALID_ARG,
                "coeff must be finite and >= 0 (got %g)", coeff);
    KBM_REQUIRE(std::isfinite(n_sigma) && n_sigma >= 0.0, KBM_ERR_INVALID_ARG,
                "n_sigma must be finite and >= 0 (got %g)", n_sigma);
    return KBM_OK;
}

RankTable make_rank_table(double q_lo, double q_hi) {
    RankTable rt{};
    for (int n = 1; n <= KBM_MAX_EPOCHS; ++n) {
        const double m = (double)(n - 1);
        rt.lo[n] = (uint8_t)std::floor(q_lo * m + 0.5);
        rt.md[n] = (uint8_t)std::floor(0.5 * m + 0.5);
        rt.hi[n] = (uint8_t)std::floor(q_hi * m + 0.5);
    }
    return rt;
}

// Pinned staging for small host tables (offsets).  One buffer per device;
// before it is overwritten, the event recorded after its previous copy is
// waited on, so an in-flight asynchronous copy never reads a reused buffer.
namespace {
struct Staging {
    void *host = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool pending = false;
};
std::mutex g_stage_mutex;
std::map<int, Staging> g_stage;
}  // namespace

kbm_status stage_to_device(void *dst, const void *src, size_t bytes,
                           hipStream_t stream) {
    if (bytes == 0) return KBM_OK;
    int dev = 0;
    KBM_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_stage_mutex);
    Staging &s = g_stage[dev];
    if (s.ev == nullptr) KBM_HIP(hipEventCreateWithFlags(&s.ev, hipEventDisableTiming));
    if (s.pending) {
        KBM_HIP(hipEventSynchronize(s.ev));
        s.pending = false;
    }
    if (bytes > s.cap) {
        if (s.host) KBM_HIP(hipHostFree(s.host));
        s.host = nullptr;
        s.cap = 0;
        const size_t cap = align_up(bytes, 1 << 20);
        KBM_HIP(hipHostMalloc(&s.host, cap, hipHostMallocDefault));
        s.cap = cap;
    }
    std::memcpy(s.host, src, bytes);
    KBM_HIP(hipMemcpyAsync(dst, s.host, bytes, hipMemcpyHostToDevice, stream));
    KBM_HIP(hipEventRecord(s.ev, stream));
    s.pending = true;
    return KBM_OK;
}

}  // namespace kbm

namespace {

// Inverse error function in double: Winitzki's closed-form approximation
// (a = 0.147) as the start, refined by Newton steps on std::erf.
double inverse_erf(double y) {
    if (y == 0.0) return 0.0;
    const double a = 0.147, pi = 3.14159265358979323846;
    const double l = std::log((1.0 - y) * (1.0 + y));
    const double b = 2.0 / (pi * a) + 0.5 * l;
    double x = std::copysign(std::sqrt(std::sqrt(b * b - l / a) - b), y);
    for (int it = 0; it < 6; ++it) {
        const double f = std::erf(x) - y;
        const double d = 2.0 / std::sqrt(pi) * std::exp(-x * x);
        const double step = f / d;
        x -= step;
        if (std::fabs(step) <= 1e-17 * std::fabs(x)) break;
    }
    return x;
}

}  // namespace

extern "C" {

kbm_status kbm_sigmag_coeff(double q_lo, double q_hi, double *coeff) {
    kbm::clear_error();
    KBM_REQUIRE(coeff != nullptr, KBM_ERR_INVALID_ARG, "kbm_sigmag_coeff: coeff is NULL");
    KBM_REQUIRE(std::isfinite(q_lo) && std::isfinite(q_hi) && q_lo > 0.0 && q_lo < q_hi &&
                    q_hi < 1.0,
                KBM_ERR_INVALID_ARG, "kbm_sigmag_coeff: need 0 < q_lo < q_hi < 1 (got %g, %g)",
                q_lo, q_hi);
    const double d = inverse_erf(2.0 * q_hi - 1.0) - inverse_erf(2.0 * q_lo - 1.0);
    *coeff = 1.0 / (std::sqrt(2.0) * d);
    return KBM_OK;
}

const char *kbm_status_string(kbm_status s) {
    switch (s) {
        case KBM_OK: return "ok";
        case KBM_ERR_INVALID_ARG: return "invalid argument";
        case KBM_ERR_UNSUPPORTED: return "unsupported";
        case KBM_ERR_OUT_OF_MEMORY: return "out of memory";
        case KBM_ERR_DEVICE: return "device error";
        case KBM_ERR_WORKSPACE: return "workspace too small";
    }
    return "unknown status";
}

const char *kbm_last_error(void) { return kbm::g_last_error.c_str(); }

int kbm_version(void) { return 100; }  // 0.1.0

#ifndef KBM_BUILD_ID
#define KBM_BUILD_ID "unknown"
#endif
const char *kbm_build_id(void) { return KBM_BUILD_ID; }

}  // extern "C"
