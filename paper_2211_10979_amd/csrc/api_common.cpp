// Entry points shared by every solver form: errors, options, sizes.
#include <string>

#include "common.hpp"

namespace lpgpu {

namespace {
thread_local std::string g_last_error;
}

int set_error(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

Options resolve_options(const lp_options *opt) {
    lp_options o;
    lp_options_default(&o);
    if (opt) o = *opt;
    Options r{};
    lp_tuning_default(&r);
    if (o.tuning) static_cast<lp_tuning &>(r) = *o.tuning;
    r.eps_dual = o.eps_dual;
    r.eps_pivot = o.eps_pivot;
    r.max_pivots = o.max_pivots;
    r.record_pivots = o.record_pivots;
    r.stream = o.stream;
    r.device_buffer = o.device_buffer;
    r.device_buffer_bytes = o.device_buffer_bytes;
    r.device = o.device;
    r.bland_after = o.bland_after;
    return r;
}

}  // namespace lpgpu

extern "C" {

const char *lp_version(void) { return "lpgpu 0.1.0 (gfx950, binary64 full-tableau simplex)"; }

const char *lp_error_string(int code) {
    switch (code) {
        case LP_OK: return "ok";
        case LP_E_INVAL: return "invalid argument";
        case LP_E_NEG_RHS: return "negative right-hand side (slack basis infeasible)";
        case LP_E_NOMEM: return "out of memory";
        case LP_E_DEVICE: return "device error";
        case LP_E_STATE: return "call out of order";
        case LP_E_PENDING: return "result pending";
        case LP_E_BUDGET: return "LP exceeds the memory budget";
        default: return "unknown code";
    }
}

const char *lp_last_error(void) { return lpgpu::g_last_error.c_str(); }

int lp_options_default(lp_options *o) {
    if (!o) return LP_E_INVAL;
    o->eps_dual = 1e-9;
    o->eps_pivot = 1e-9;
    o->max_pivots = 0;
    o->record_pivots = 1;
    o->stream = nullptr;
    o->device_buffer = nullptr;
    o->device_buffer_bytes = 0;
    o->device = 0;
    o->bland_after = 0;
    o->tuning = nullptr;
    return LP_OK;
}

int lp_tuning_default(lp_tuning *t) {
    if (!t) return LP_E_INVAL;
    *t = lp_tuning{};
    return LP_OK;
}

size_t lp_tableau_bytes(int32_t m, int32_t n) {
    if (m < 1 || n < 1) return 0;
    return (size_t)lpgpu::padded_ld(m) * ((size_t)n + (size_t)m + 1) * sizeof(double);
}

}  // extern "C"
