// hc_api.cpp -- host side of the C ABI declared in include/hc.h.
//
// Owns contexts, loaded systems (their kernel tables on the device), the device
// workspace that holds the structure-of-arrays path state, and the launch
// sequence prep -> init -> track (FP32 pass + FP64 pass in mixed mode) -> refine.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "hc_host.h"

using namespace hcx;

namespace hcx {

namespace {
thread_local std::string g_err;
}

hc_status fail(hc_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

void clear_error() { g_err.clear(); }

const char *last_error() { return g_err.c_str(); }

namespace {

template <typename T>
hipError_t upload(T **dst, const T *src, size_t count)
{
    *dst = nullptr;
    if (count == 0) return hipSuccess;
    hipError_t e = hipMalloc((void **)dst, count * sizeof(T));
    if (e != hipSuccess) return e;
    return hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice);
}

}  // namespace
}  // namespace hcx

extern "C" {

void hc_default_opts(hc_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->h0 = 0.05;
    o->h_min = 1e-7;
    o->h_max = 0.1;
    o->beta_inc = 2.0;
    o->beta_dec = 0.5;
    o->tau64 = 1e-6;
    o->tau32 = 3e-4;
    o->pred_tol = 1e-2;
    o->tau_refine = 1e-14;
    o->inf_bound = 1e7;
    o->eta_max = 1e-10;
    o->t_end = 0.0;
    o->precision = HC_FP64;
    o->n_inc = 5;
    o->max_newton = 3;
    o->max_steps = 5000;
    o->max_refine = 10;
    o->steps_per_launch = 0;
    o->tracks_per_item = 0;
    o->lanes_per_path = 0;
    o->fp64_residual = 0;
    o->crossing_check = 1;
    o->per_instance_start = 0;
    o->endgame = 0;
    o->eg_max_newton = 5;
    o->eg_max_samples = 16;
    o->eg_max_cycle = 8;
    o->eg_s0 = 0.1;
    o->eg_beta = 0.25;
    o->eg_tol = 1e-9;
    o->eg_tol_inf = 1e-3;
    o->eg_tau = 1e-8;
    o->eg_h_min = 1e-14;
}

const char *hc_last_error(void) { return last_error(); }

hc_status hc_create(int device, hc_ctx **out)
{
    clear_error();
    if (!out) return fail(HC_E_INVALID, "hc_create: out is NULL");
    int count = 0;
    HIP_TRY(hipGetDeviceCount(&count));
    if (device < 0 || device >= count)
        return fail(HC_E_INVALID, "hc_create: device %d not in [0, %d)", device, count);
    HIP_TRY(hipSetDevice(device));
    hc_ctx *c = new (std::nothrow) hc_ctx;
    if (!c) return fail(HC_E_OOM, "hc_create: out of host memory");
    c->device = device;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, device);
    if (e == hipSuccess) {
        c->arch = prop.gcnArchName;
        c->arch = c->arch.substr(0, c->arch.find(':'));  // gfx950, without feature flags
        e = hipStreamCreate(&c->own_stream);
    }
    // the no-allocation entry point's workspace: its address on this device,
    // looked up once per device
    if (e == hipSuccess) e = scratch_init(device);
    if (e != hipSuccess) {
        delete c;
        return fail(HC_E_DEVICE, "hc_create: %s", hipGetErrorString(e));
    }
    // a persisted autotuner cache, if HC_TUNE_CACHE names one (a missing file is
    // created by the first hc_autotune)
    if (const char *f = std::getenv("HC_TUNE_CACHE")) {
        c->tune_file = f;
        int32_t loaded = 0;
        std::ifstream probe(c->tune_file);
        if (probe.good() && hc_tune_load(c, f, &loaded) != HC_OK) {
            hc_destroy(c);
            return fail(HC_E_INVALID, "hc_create: HC_TUNE_CACHE file %s is malformed", f);
        }
    }
    *out = c;
    return HC_OK;
}

static void free_system_tables(hc_system *s)
{
    if (s->alt) {
        free_system_tables(s->alt);
        delete s->alt;
        s->alt = nullptr;
    }
    (void)hipFree(s->d_slot_ptr);
    (void)hipFree(s->d_slot_term);
    (void)hipFree(s->d_slot_mult);
    (void)hipFree(s->d_term_const);
    (void)hipFree(s->d_map_ptr);
    (void)hipFree(s->d_map_col);
    (void)hipFree(s->d_map_val);
    (void)hipFree(s->d_vars);
    (void)hipFree(s->d_sdeg);
    (void)hipFree(s->d_eqdeg);
}

void hc_destroy(hc_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (hc_system *s : c->systems) {
        free_system_tables(s);
        delete s;
    }
    c->state.release();
    c->coef.release();
    c->io.release();
    c->counter.release();
    c->queue.release();
    c->eg.release();
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->bgraph_exec) (void)hipGraphExecDestroy(c->bgraph_exec);
    for (hipEvent_t &e : c->ev)
        if (e) (void)hipEventDestroy(e);
    if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
    delete c;
}

hc_status hc_load_system(hc_ctx *c, const hc_system_desc *d, hc_system **out)
{
    return hc_load_system_layout(c, d, HC_LAYOUT_AUTO, out);
}

}  // extern "C"

// Validates a description and uploads its tables in `layout`; the system is
// added to the context's list when `owned` (else its caller owns it: the
// autotuner's copy in the other layout).
static hc_status load_system_impl(hc_ctx *c, const hc_system_desc *d, int32_t layout, bool owned, hc_system **out)
{
    if (!c || !d || !out) return fail(HC_E_INVALID, "hc_load_system: NULL argument");
    if (d->n < 1) return fail(HC_E_INVALID, "hc_load_system: n = %d", d->n);
    if (d->n > HC_MAX_N) return fail(HC_E_UNSUPPORTED, "hc_load_system: n = %d > %d", d->n, HC_MAX_N);
    if (d->n_terms < 1 || !d->term_eq || !d->term_exp)
        return fail(HC_E_INVALID, "hc_load_system: empty or missing term tables");
    if (d->kind != HC_TOTAL_DEGREE && d->kind != HC_PARAMETER)
        return fail(HC_E_INVALID, "hc_load_system: kind = %d", d->kind);
    if (d->n_params < 0) return fail(HC_E_INVALID, "hc_load_system: n_params = %d", d->n_params);
    const int n = d->n, nt = d->n_terms;
    // degrees of the terms (validated before the layout is chosen)
    std::vector<int> tdeg(nt, 0);
    int max_deg = 0;
    for (int k = 0; k < nt; k++) {
        if (d->term_eq[k] < 0 || d->term_eq[k] >= n)
            return fail(HC_E_INVALID, "hc_load_system: term_eq[%d] = %d out of range", k, d->term_eq[k]);
        for (int j = 0; j < n; j++) {
            const int e = d->term_exp[(size_t)k * n + j];
            if (e < 0) return fail(HC_E_INVALID, "hc_load_system: negative exponent in term %d", k);
            if (e > kMaxTermDeg)
                return fail(HC_E_UNSUPPORTED, "hc_load_system: term %d has degree > %d", k, kMaxTermDeg);
            tdeg[k] += e;
        }
        if (tdeg[k] > kMaxTermDeg)
            return fail(HC_E_UNSUPPORTED, "hc_load_system: term %d has degree %d > %d", k, tdeg[k], kMaxTermDeg);
        max_deg = std::max(max_deg, tdeg[k]);
    }
    if (layout == HC_LAYOUT_AUTO) layout = (n <= 8 && max_deg <= 2) ? HC_LAYOUT_DENSE : HC_LAYOUT_TERMS;
    if (layout != HC_LAYOUT_DENSE && layout != HC_LAYOUT_TERMS)
        return fail(HC_E_UNSUPPORTED, "hc_load_system: layout %d", layout);
    if (layout == HC_LAYOUT_DENSE && n > 8)
        return fail(HC_E_UNSUPPORTED, "hc_load_system: dense tables need n <= 8 (n = %d)", n);
    if (layout == HC_LAYOUT_DENSE && max_deg > 2)
        return fail(HC_E_UNSUPPORTED, "hc_load_system: dense tables need degree <= 2 (a term has degree %d)",
                    max_deg);
    if (layout == HC_LAYOUT_TERMS && n < 2)
        return fail(HC_E_UNSUPPORTED, "hc_load_system: term lists need n >= 2");
    // term-list kernel kind: the quadratic kernels where they apply
    const int tk = layout != HC_LAYOUT_TERMS ? 0 : term_kind_for(max_deg, n);
    const bool gen = layout == HC_LAYOUT_TERMS && term_kind_general(tk);
    if (!d->coef_rowptr && d->n_params != nt)
        return fail(HC_E_INVALID, "hc_load_system: identity coefficient map needs n_params == n_terms (%d != %d)",
                    d->n_params, nt);
    int nnz = 0;
    if (d->coef_rowptr) {
        if (d->coef_rowptr[0] != 0) return fail(HC_E_INVALID, "hc_load_system: coef_rowptr[0] != 0");
        for (int k = 0; k < nt; k++)
            if (d->coef_rowptr[k + 1] < d->coef_rowptr[k])
                return fail(HC_E_INVALID, "hc_load_system: coef_rowptr decreases at %d", k);
        nnz = d->coef_rowptr[nt];
        if (nnz > 0 && (!d->coef_col || !d->coef_val))
            return fail(HC_E_INVALID, "hc_load_system: coef_col/coef_val missing");
        for (int e = 0; e < nnz; e++)
            if (d->coef_col[e] < 0 || d->coef_col[e] >= d->n_params)
                return fail(HC_E_INVALID, "hc_load_system: coef_col[%d] = %d out of range", e, d->coef_col[e]);
    }

    hc_system *s = new (std::nothrow) hc_system;
    if (!s) return fail(HC_E_OOM, "hc_load_system: out of host memory");
    s->device = c->device;
    s->n = n;
    s->n_terms = nt;
    s->n_params = d->n_params;
    s->kind = d->kind;
    s->layout = layout;
    s->tk = tk;
    s->max_deg = max_deg;
    s->deg.assign(n, 0);
    for (int k = 0; k < nt; k++) s->deg[d->term_eq[k]] = std::max(s->deg[d->term_eq[k]], tdeg[k]);
    // term lists: slot j of equation i is its j-th term; the general-degree kinds
    // order each equation's terms by decreasing degree (stable)
    std::vector<int> eq_count(n, 0), term_pos(nt);
    if (gen) {
        std::vector<int> order(nt);
        for (int k = 0; k < nt; k++) order[k] = k;
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return tdeg[x] > tdeg[y]; });
        for (int k : order) term_pos[k] = eq_count[d->term_eq[k]]++;
    } else {
        for (int k = 0; k < nt; k++) term_pos[k] = eq_count[d->term_eq[k]]++;
    }
    s->T = layout == HC_LAYOUT_DENSE ? dense_terms(n) : *std::max_element(eq_count.begin(), eq_count.end());

    // a0: map every term to its slot in the kernel tables
    const int n_slots = n * s->T;
    std::vector<std::vector<std::pair<int, int>>> slot_terms(n_slots);
    std::vector<unsigned short> vars((layout == HC_LAYOUT_TERMS && !gen) ? n_slots : 0, 0xFFFFu);
    std::vector<unsigned long long> vars64(gen ? n_slots : 0, ~0ull);
    std::vector<int> sdeg(gen ? s->T : 0, 0);
    for (int k = 0; k < nt; k++) {
        const int i = d->term_eq[k];
        const int deg = tdeg[k];
        if (gen) {
            // factor bytes, variables in increasing order with repetition
            const int q = i * s->T + term_pos[k];
            unsigned long long v = ~0ull;
            int f = 0;
            for (int j = 0; j < n; j++)
                for (int e = 0; e < d->term_exp[(size_t)k * n + j]; e++, f++)
                    v = (v & ~(0xFFull << (8 * f))) | ((unsigned long long)j << (8 * f));
            vars64[q] = v;
            sdeg[term_pos[k]] = std::max(sdeg[term_pos[k]], deg);
            slot_terms[q].push_back({k, 1});
            continue;
        }
        int a = -1, b = -1;
        for (int j = 0; j < n; j++)
            for (int e = 0; e < d->term_exp[(size_t)k * n + j]; e++) {
                if (a < 0) a = j;
                else b = j;
            }
        if (layout == HC_LAYOUT_TERMS) {
            // c x_a x_b with 0xFF for a missing factor
            const int q = i * s->T + term_pos[k];
            vars[q] = (unsigned short)((a < 0 ? 0xFFu : (unsigned)a) | ((b < 0 ? 0xFFu : (unsigned)b) << 8));
            slot_terms[q].push_back({k, 1});
            continue;
        }
        int slot, mult = 1;
        if (deg == 0) slot = 0;
        else if (deg == 1) slot = 1 + a;
        else {
            if (b < 0) b = a;
            if (a > b) std::swap(a, b);
            slot = quad_slot(n, a, b);
            if (a == b) mult = 2;  // x_a^2 enters dF/dx_a twice
        }
        slot_terms[(size_t)i * s->T + slot].push_back({k, mult});
    }
    int64_t bez = 1;
    for (int i = 0; i < n; i++) {
        if (s->deg[i] < 1) {
            delete s;
            return fail(HC_E_UNSUPPORTED, "hc_load_system: equation %d has degree 0", i);
        }
        if (s->deg[i] == 2) s->deg2 |= 1u << i;
        bez = bez > (int64_t)(INT64_MAX / s->deg[i]) ? INT64_MAX : bez * s->deg[i];
    }
    s->bezout = bez;
    std::vector<int> slot_ptr(n_slots + 1, 0), slot_term, slot_mult;
    for (int q = 0; q < n_slots; q++) {
        slot_ptr[q + 1] = slot_ptr[q] + (int)slot_terms[q].size();
        for (auto &pr : slot_terms[q]) {
            slot_term.push_back(pr.first);
            slot_mult.push_back(pr.second);
        }
    }

    hipError_t e = hipSetDevice(c->device);
    if (e == hipSuccess) e = upload(&s->d_slot_ptr, slot_ptr.data(), slot_ptr.size());
    if (e == hipSuccess) e = upload(&s->d_slot_term, slot_term.data(), slot_term.size());
    if (e == hipSuccess) e = upload(&s->d_slot_mult, slot_mult.data(), slot_mult.size());
    if (e == hipSuccess && !vars.empty()) {
        unsigned short *dv = nullptr;
        e = upload(&dv, vars.data(), vars.size());
        s->d_vars = dv;
    }
    if (e == hipSuccess && !vars64.empty()) {
        unsigned long long *dv = nullptr;
        e = upload(&dv, vars64.data(), vars64.size());
        s->d_vars = dv;
        if (e == hipSuccess) e = upload(&s->d_sdeg, sdeg.data(), sdeg.size());
        if (e == hipSuccess) e = upload(&s->d_eqdeg, s->deg.data(), s->deg.size());
    }
    if (e == hipSuccess && d->coef_const) {
        s->has_const = true;
        e = upload(&s->d_term_const, reinterpret_cast<const double *>(d->coef_const), (size_t)nt * 2);
    }
    if (e == hipSuccess && d->coef_rowptr) {
        s->has_map = true;
        e = upload(&s->d_map_ptr, d->coef_rowptr, (size_t)nt + 1);
        if (e == hipSuccess) e = upload(&s->d_map_col, d->coef_col, (size_t)nnz);
        if (e == hipSuccess) e = upload(&s->d_map_val, reinterpret_cast<const double *>(d->coef_val), (size_t)nnz * 2);
    }
    if (e != hipSuccess) {
        free_system_tables(s);
        delete s;
        return fail(e == hipErrorOutOfMemory ? HC_E_OOM : HC_E_DEVICE, "hc_load_system: %s", hipGetErrorString(e));
    }
    // host copy of the description
    s->h_term_eq.assign(d->term_eq, d->term_eq + nt);
    s->h_term_exp.assign(d->term_exp, d->term_exp + (size_t)nt * n);
    if (d->coef_const) s->h_const.assign(d->coef_const, d->coef_const + nt);
    if (d->coef_rowptr) {
        s->h_rowptr.assign(d->coef_rowptr, d->coef_rowptr + nt + 1);
        s->h_col.assign(d->coef_col, d->coef_col + nnz);
        s->h_val.assign(d->coef_val, d->coef_val + nnz);
    }
    if (owned) c->systems.push_back(s);
    *out = s;
    return HC_OK;
}

// The system in the other table layout (dense tables <-> term lists), loaded
// from its stored description on first use; null if that layout cannot hold it.
static hc_system *alt_layout(hc_ctx *c, const hc_system *s)
{
    if (s->alt) return s->alt;
    const int other = s->layout == HC_LAYOUT_DENSE ? HC_LAYOUT_TERMS : HC_LAYOUT_DENSE;
    if (other == HC_LAYOUT_DENSE && (s->n > 8 || s->max_deg > 2)) return nullptr;
    if (other == HC_LAYOUT_TERMS && s->n < 2) return nullptr;
    hc_system_desc d{};
    d.n = s->n;
    d.n_terms = s->n_terms;
    d.term_eq = s->h_term_eq.data();
    d.term_exp = s->h_term_exp.data();
    d.n_params = s->n_params;
    d.kind = s->kind;
    d.coef_const = s->h_const.empty() ? nullptr : s->h_const.data();
    d.coef_rowptr = s->h_rowptr.empty() ? nullptr : s->h_rowptr.data();
    d.coef_col = s->h_col.empty() ? nullptr : s->h_col.data();
    d.coef_val = s->h_val.empty() ? nullptr : s->h_val.data();
    hc_system *a = nullptr;
    if (load_system_impl(c, &d, other, false, &a) != HC_OK) return nullptr;
    const_cast<hc_system *>(s)->alt = a;
    return a;
}

extern "C" {

hc_status hc_load_system_layout(hc_ctx *c, const hc_system_desc *d, int32_t layout, hc_system **out)
{
    clear_error();
    return load_system_impl(c, d, layout, true, out);
}

hc_status hc_free_system(hc_ctx *c, hc_system *s)
{
    clear_error();
    if (!c || !s) return fail(HC_E_INVALID, "hc_free_system: NULL argument");
    auto it = std::find(c->systems.begin(), c->systems.end(), s);
    if (it == c->systems.end()) return fail(HC_E_INVALID, "hc_free_system: system not owned by this context");
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    free_system_tables(s);
    delete s;
    c->systems.erase(it);
    c->graph_valid = false;
    c->bgraph_valid = false;
    return HC_OK;
}

hc_status hc_system_dims(const hc_system *s, int32_t *n, int64_t *bezout)
{
    clear_error();
    if (!s) return fail(HC_E_INVALID, "hc_system_dims: NULL system");
    if (n) *n = s->n;
    if (bezout) *bezout = s->bezout;
    return HC_OK;
}

hc_status hc_total_degree_start(const hc_system *s, int64_t first, int64_t count, hc_c64 *out)
{
    clear_error();
    if (!s || (count > 0 && !out)) return fail(HC_E_INVALID, "hc_total_degree_start: NULL argument");
    if (first < 0 || count < 0 || first + count > s->bezout)
        return fail(HC_E_INVALID, "hc_total_degree_start: range [%lld, %lld) outside [0, %lld)",
                    (long long)first, (long long)(first + count), (long long)s->bezout);
    const double two_pi = 6.283185307179586476925286766559;
    for (int64_t q = 0; q < count; q++) {
        int64_t r = first + q;
        for (int i = 0; i < s->n; i++) {
            const int d = s->deg[i];
            const int64_t j = r % d;
            r /= d;
            hc_c64 v;
            if (j == 0) v = {1.0, 0.0};
            else if (2 * j == d) v = {-1.0, 0.0};
            else v = {std::cos(two_pi * (double)j / d), std::sin(two_pi * (double)j / d)};
            out[q * s->n + i] = v;
        }
    }
    return HC_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ tracking

static hc_status check_opts(const hc_opts &o)
{
    if (o.per_instance_start != 0 && o.per_instance_start != 1)
        return fail(HC_E_INVALID, "opts.per_instance_start = %d", o.per_instance_start);
    if (o.precision != HC_FP64 && o.precision != HC_MIXED)
        return fail(HC_E_INVALID, "opts.precision = %d", o.precision);
    if (!(o.h0 > 0) || !(o.h_max > 0) || !(o.h_min >= 0) || !(o.beta_dec > 0 && o.beta_dec < 1) ||
        !(o.beta_inc >= 1) || o.n_inc < 1 || o.max_newton < 0 || o.max_steps < 0 || o.max_refine < 0 ||
        o.steps_per_launch < -1 || o.tracks_per_item < 0)
        return fail(HC_E_INVALID, "opts: step-control values out of range");
    if (o.table_layout != HC_LAYOUT_AUTO && o.table_layout != HC_LAYOUT_DENSE && o.table_layout != HC_LAYOUT_TERMS)
        return fail(HC_E_INVALID, "opts.table_layout = %d", o.table_layout);
    if (o.lanes_per_path != 0 && o.lanes_per_path != 1 && o.lanes_per_path != 4 && o.lanes_per_path != 8 &&
        o.lanes_per_path != 16 && o.lanes_per_path != 64)
        return fail(HC_E_INVALID, "opts.lanes_per_path = %d (0, 1, 4, 8, 16 or 64)", o.lanes_per_path);
    if (o.precision == HC_MIXED && !(o.t_end >= 0 && o.t_end < 1))
        return fail(HC_E_INVALID, "opts.t_end = %g must lie in [0, 1) in mixed mode", o.t_end);
    if (o.endgame < 0 || o.endgame > 2) return fail(HC_E_INVALID, "opts.endgame = %d (0, 1 or 2)", o.endgame);
    if (o.endgame &&
        (!(o.eg_s0 > 0 && o.eg_s0 < 1) || !(o.eg_beta > 0 && o.eg_beta < 1) || !(o.eg_tol > 0) ||
         !(o.eg_tol_inf >= 0) || !(o.eg_tau > 0) || !(o.eg_h_min >= 0) || o.eg_max_newton < 1 ||
         o.eg_max_samples < 0 || o.eg_max_samples > kEgMaxSamples || o.eg_max_cycle < 1))
        return fail(HC_E_INVALID, "opts: end-game values out of range");
    return HC_OK;
}

// Batch path: one device queue per [dense | term-list kind] x [total degree |
// parameter], and one refinement launch per dense n and per term-list kind.
constexpr int kQueues = 2 + 2 * kTermKindCount;
constexpr int kRefSlots = kMaxN + 1 + kTermKindCount;

// Lanes per path: one row of [H_x | rhs] per lane (dense tables: G = 4 for
// n <= 4, 8 for n <= 8; term lists: 16, or 32 for n > 16) unless one path per
// lane is asked for (dense tables) or n = 1.  -1: the option does not fit the
// system.
// The one-path-per-wavefront tracker (hc_wave.hip) holds dense total-degree
// systems with 2 <= n <= 8 in FP64.
static bool wave_fits(const hc_system *s)
{
    return s->layout == HC_LAYOUT_DENSE && s->kind == HC_TOTAL_DEGREE && s->n >= 2 && s->n <= 8;
}

// Mixed precision on the single-call group trackers: failed FP32 paths go on in
// FP64 inside the FP32 launch (dense tables, g16), or in a second, FP64 launch
// (the other term-list kinds).  The batch tracker always escalates inline.
static bool inline_escalation(const hc_system *s)
{
    return kInlineEsc && (s->layout != HC_LAYOUT_TERMS || term_kind_inline_esc(s->tk));
}

static int choose_lanes_per_path(const hc_opts &o, const hc_system *s)
{
    if (o.lanes_per_path == 64) return wave_fits(s) && o.precision == HC_FP64 ? 64 : -1;
    if (s->layout == HC_LAYOUT_TERMS) {
        const int g = term_kind_lanes(s->tk);
        return (o.lanes_per_path == 0 || o.lanes_per_path == g) ? g : -1;
    }
    if (s->n < 2) return 1;
    if (o.lanes_per_path == 1) return 1;
    const int g = group_lanes(s->n);
    if (o.lanes_per_path != 0 && o.lanes_per_path != g && o.lanes_per_path < g) return -1;  // too few lanes
    if (o.lanes_per_path == 16) return -1;
    return g;
}

static int lanes_for(const hc_system *s)
{
    return s->layout == HC_LAYOUT_TERMS ? term_kind_lanes(s->tk) : group_lanes(s->n);
}

// Term lists of the general-degree kinds carry their equations' degrees (start
// system and start points of any degree).
static const int *eqdeg_of(const hc_system *s) { return s->layout == HC_LAYOUT_TERMS ? s->d_eqdeg : nullptr; }
static const int *sdeg_of(const hc_system *s) { return s->layout == HC_LAYOUT_TERMS ? s->d_sdeg : nullptr; }

// Paths per work item.  Group layouts pop items from a device counter, so small
// items balance the wavefronts (measured best: 1 path per lane group); the
// one-path-per-lane layout has fixed items of 64 paths.
static int choose_tracks_per_item(const hc_opts &o, int n_start, int lanes)
{
    if (o.tracks_per_item > 0) return o.tracks_per_item;
    const int slots = 64 / lanes;
    return std::max(1, std::min(n_start, lanes == 1 ? 64 : slots));
}

template <typename T>
static void put(std::vector<unsigned char> &k, const T &v)
{
    const unsigned char *b = reinterpret_cast<const unsigned char *>(&v);
    k.insert(k.end(), b, b + sizeof(T));
}

// Autotuner key: the workload's shape, not the system's address (a system loaded
// later with the same shape takes the same choice; a freed one leaves nothing
// behind that could mislead a new one).
static std::string tune_key(const hc_ctx *c, const hc_system *s, int precision, int n_start, int n_inst)
{
    char b[256];
    std::snprintf(b, sizeof b, "%s layout=%d kind=%d n=%d terms=%d slots=%d maxdeg=%d deg2=%x tk=%d prec=%d "
                  "n_start=%d n_inst=%d", c->arch.c_str(), s->layout, s->kind, s->n, s->n_terms, s->T, s->max_deg,
                  s->deg2, s->tk, precision, n_start, n_inst);
    return b;
}

// Applies a tuned choice for this workload when the call leaves the work
// decomposition to the library (tracks_per_item = lanes_per_path = 0; a
// steps_per_launch of -1 takes the tuned value too, else 0).  May switch the
// system to its copy in the tuned table layout.
static hc_status apply_tuning(hc_ctx *c, const hc_system *&s, hc_opts &o, int n_start, int n_inst,
                              bool may_alloc = true)
{
    if (o.lanes_per_path == 0 && o.tracks_per_item == 0 && o.table_layout == HC_LAYOUT_AUTO) {
        auto it = c->tune.find(tune_key(c, s, o.precision, n_start, n_inst));
        if (it != c->tune.end()) {
            const TuneChoice &tc = it->second;
            o.table_layout = tc.layout;
            o.lanes_per_path = tc.lanes;
            o.tracks_per_item = tc.tpi;
            if (o.steps_per_launch < 0) o.steps_per_launch = tc.spl;
        }
    }
    if (o.steps_per_launch < 0) o.steps_per_launch = 0;
    if (o.table_layout != HC_LAYOUT_AUTO && o.table_layout != s->layout) {
        if (!may_alloc && !s->alt)
            return fail(HC_E_UNSUPPORTED, "table_layout = %d needs a copy of the system in that layout, "
                        "which the no-allocation entry point does not make", o.table_layout);
        const hc_system *t = alt_layout(c, s);
        if (!t || t->layout != o.table_layout)
            return fail(HC_E_UNSUPPORTED, "opts.table_layout = %d cannot hold this system (n = %d, degree %d)",
                        o.table_layout, s->n, s->max_deg);
        s = t;
    }
    return HC_OK;
}

// Mixed mode with the crossing check on instances above kDedupMax paths: the
// check keeps its projections in the workspace (16 bytes per path).
static bool mixed_check_big(const hc_opts &o, int n_start)
{
    return o.precision == HC_MIXED && o.crossing_check && n_start > kDedupMax;
}

static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

// The power-series end-game after refinement (opts.endgame): candidates (paths
// that failed in the zone [1 - eg_s0, 1], or every path there with endgame = 2)
// are compacted into a list and re-tracked in FP64 from their start points to
// 1 - eg_s0 with the usual options, then with the zone's options to 1 - s_k for
// k = 1 .. eg_max_samples, one launch per sample followed by k_eg_sample.  Paths
// it classifies at infinity are written out by k_eg_sample; finite estimates
// with cycle number 1 get the usual refinement, those with cycle number >= 2
// only the classification (HC_T_SINGULAR_END).  Candidates whose end-game does
// not converge keep the outputs of the first refinement.  Needs one host
// round trip (the candidate count) and an allocation for the candidates.
template <typename RunPass>
static hc_status run_endgame(hc_ctx *c, const hc_system *s, hc_opts &o, long long total, const TrackState &S,
                             const InitArgs &ia, const RefineArgs &ra, char *counter_p, RunPass &run_pass,
                             TrackArgs &ta, hipStream_t st)
{
    EgArgs ea{};
    ea.n = s->n;
    ea.total = total;
    ea.s = S;
    ea.mode = o.endgame;
    ea.s0 = o.eg_s0;
    ea.beta = o.eg_beta;
    ea.tol = o.eg_tol;
    ea.tol_inf = o.eg_tol_inf;
    ea.inf_bound = o.inf_bound;
    ea.max_cycle = o.eg_max_cycle;
    ea.endpoints = ra.endpoints;
    ea.status = ra.status;
    ea.info = ra.info;
    ea.count = reinterpret_cast<unsigned *>(counter_p + 48);
    HIP_TRY(c->eg.ensure((size_t)total * sizeof(int)));
    ea.list = static_cast<int *>(c->eg.p);
    HIP_TRY(launch_fill_u32(ea.count, 0u, 1, st));
    HIP_TRY(launch_eg_select(ea, st));
    unsigned m = 0;
    HIP_TRY(hipMemcpyAsync(&m, ea.count, sizeof m, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (m == 0) return HC_OK;
    // per candidate: 3 samples + the previous estimate (n + 1 complex each), class, flag
    const size_t n1 = (size_t)s->n + 1;
    const size_t list_b = al256((size_t)total * sizeof(int));
    const size_t ring_b = al256((size_t)3 * m * n1 * 16), prev_b = al256((size_t)m * n1 * 16);
    const size_t need = list_b + ring_b + prev_b + 2 * al256((size_t)m * sizeof(int));
    if (need > c->eg.cap) {
        // grow, keeping the candidate list
        std::vector<int> keep(m);
        HIP_TRY(hipMemcpyAsync(keep.data(), c->eg.p, (size_t)m * sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        HIP_TRY(c->eg.ensure(need));
        HIP_TRY(hipMemcpyAsync(c->eg.p, keep.data(), (size_t)m * sizeof(int), hipMemcpyHostToDevice, st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    char *base = static_cast<char *>(c->eg.p);
    ea.list = reinterpret_cast<int *>(base);
    ea.ring = reinterpret_cast<double *>(base + list_b);
    ea.prev = reinterpret_cast<double *>(base + list_b + ring_b);
    ea.cls = reinterpret_cast<int *>(base + list_b + ring_b + prev_b);
    ea.have_prev = reinterpret_cast<int *>(base + list_b + ring_b + prev_b + al256((size_t)m * sizeof(int)));
    ea.m = (int)m;
    HIP_TRY(launch_fill_u32(reinterpret_cast<unsigned *>(ea.cls), 0u, (int)m, st));
    HIP_TRY(launch_fill_u32(reinterpret_cast<unsigned *>(ea.have_prev), 0u, (int)m, st));

    // re-track the candidates in FP64 to the zone with the usual options
    InitArgs ir = ia;
    ir.retrack = 1;
    HIP_TRY(launch_init(ir, st));
    hc_status rc = run_pass(false, 1.0 - o.eg_s0, 0, true);
    if (rc != HC_OK) return rc;
    // inside the zone: the end-game's corrector and minimum step
    const double tau64 = o.tau64, h_min = ta.h_min;
    const int max_newton = ta.max_newton;
    o.tau64 = o.eg_tau;
    ta.h_min = o.eg_h_min;
    ta.max_newton = o.eg_max_newton;
    double sk = o.eg_s0;
    for (int k = 1; k <= o.eg_max_samples && rc == HC_OK; k++) {
        sk *= o.eg_beta;
        ea.k = k;
        ea.t_k = 1.0 - sk;
        rc = run_pass(false, ea.t_k, 0, true);
        if (rc == HC_OK) {
            const hipError_t e = launch_eg_sample(ea, st);
            if (e != hipSuccess) rc = fail(HC_E_DEVICE, "launch_eg_sample: %s", hipGetErrorString(e));
        }
    }
    o.tau64 = tau64;
    ta.h_min = h_min;
    ta.max_newton = max_newton;
    if (rc != HC_OK) return rc;

    // cycle number 1: the usual refinement from the estimate; >= 2: classification only
    RefineArgs r1 = ra;
    r1.eg_cycle = 1;
    RefineArgs r2 = r1;
    r2.max_refine = 0;
    r2.singular_end = 1;
    for (int cls = 1; cls <= 2; cls++) {
        HIP_TRY(launch_eg_mark(ea, cls, st));
        const RefineArgs &r = cls == 1 ? r1 : r2;
        if (s->layout == HC_LAYOUT_TERMS) HIP_TRY(launch_refine_terms(s->tk, r, st));
        else HIP_TRY(launch_refine(s->n, r, st));
    }
    return HC_OK;
}

static hc_status track_device_impl(hc_ctx *c, const hc_system *s, const hc_c64 *start, int32_t n_start,
                                   const hc_c64 *p_start, const hc_c64 *p_target, int32_t n_inst,
                                   const hc_c64 *gamma, const hc_opts *opts_in, hc_c64 *endpoints,
                                   int32_t *status, hc_track_info *info, hipStream_t st,
                                   bool noalloc = false)
{
    if (!c || !s) return fail(HC_E_INVALID, "hc_track: NULL context or system");
    if (n_start < 0 || n_inst < 0) return fail(HC_E_INVALID, "hc_track: negative size");
    hc_opts o;
    if (opts_in) o = *opts_in;
    else hc_default_opts(&o);
    hc_status rc = check_opts(o);
    if (rc != HC_OK) return rc;
    rc = apply_tuning(c, s, o, n_start, n_inst, !noalloc);
    if (rc != HC_OK) return rc;
    if (noalloc && o.endgame)
        return fail(HC_E_UNSUPPORTED, "hc_track_device_noalloc: the end-game allocates its candidate buffers");
    const bool param = s->kind == HC_PARAMETER;
    if (!param && !start && n_start > s->bezout)
        return fail(HC_E_INVALID, "hc_track: n_start = %d exceeds the Bezout number %lld", n_start,
                    (long long)s->bezout);
    if (param && n_start > 0 && n_inst > 0 && (!start || (!p_start && s->n_params > 0)))
        return fail(HC_E_INVALID, "hc_track: a parameter homotopy needs start points and p_start");
    const long long total = (long long)n_start * n_inst;
    if (total == 0) return HC_OK;
    if (!p_target && s->n_params > 0) return fail(HC_E_INVALID, "hc_track: p_target is NULL");
    if (!endpoints || !status) return fail(HC_E_INVALID, "hc_track: NULL output");
    HIP_TRY(hipSetDevice(c->device));

    const int n = s->n, T = s->T;
    const bool mixed = o.precision == HC_MIXED;
    const int n_slots = n * T;

    // workspace: SoA state (+ the crossing check's projections of instances
    // above kDedupMax paths), then kernel tables
    const size_t st_doubles = (size_t)total * (2 * n + 2);
    const size_t st_ints = (size_t)total * 6;
    const bool big_check = mixed_check_big(o, n_start);
    const size_t proj_off = al256(st_doubles * 8 + st_ints * 4);
    const size_t state_core = big_check ? proj_off + (size_t)total * 16 : st_doubles * 8 + st_ints * 4;
    // dense total-degree systems: the list of paths the one-path-per-wavefront
    // tracker re-tracks (4 bytes per path)
    const size_t wave_off = al256(state_core);
    const size_t state_bytes = wave_fits(s) ? wave_off + (size_t)total * 4 : state_core;
    // tables: n_inst target instances (+ the start instance(s) of a parameter homotopy)
    const bool pis = o.per_instance_start != 0;
    const int n_tab = n_inst + (param ? (pis ? n_inst : 1) : 0);
    const size_t coef64 = (size_t)n_tab * n_slots * 2 * sizeof(double);
    const size_t coef32 = mixed ? (size_t)n_tab * n_slots * 2 * sizeof(float) : 0;
    char *state_p, *coef_p, *counter_p;
    if (noalloc) {
        // the device's fixed scratch array: counters | state | tables
        const size_t need = 256 + al256(state_bytes) + al256(coef64 + coef32);
        if (need > kScratchBytes)
            return fail(HC_E_UNSUPPORTED, "hc_track_device_noalloc: the call needs %zu workspace bytes, the "
                        "fixed workspace holds %zu", need, kScratchBytes);
        char *base = static_cast<char *>(scratch_ptr(c->device));
        if (!base) return fail(HC_E_DEVICE, "hc_track_device_noalloc: no workspace address for device %d", c->device);
        counter_p = base;
        state_p = base + 256;
        coef_p = state_p + al256(state_bytes);
    } else {
        HIP_TRY(c->state.ensure(state_bytes));
        HIP_TRY(c->coef.ensure(coef64 + coef32));
        HIP_TRY(c->counter.ensure(64));
        state_p = static_cast<char *>(c->state.p);
        coef_p = static_cast<char *>(c->coef.p);
        counter_p = static_cast<char *>(c->counter.p);
    }
    unsigned long long *stage_ctr = reinterpret_cast<unsigned long long *>(counter_p + 16);
    const bool prof = c->profiling && !noalloc;
    if (prof) {
        for (hipEvent_t &e : c->ev)
            if (!e) HIP_TRY(hipEventCreate(&e));
        HIP_TRY(hipMemsetAsync(stage_ctr, 0, 2 * sizeof(unsigned long long), st));
        HIP_TRY(hipEventRecord(c->ev[0], st));
        c->launches_fp32 = c->launches_fp64 = 0;
        c->had_fp32 = false;
    }

    TrackState S;
    double *dp = reinterpret_cast<double *>(state_p);
    S.xr = dp;
    S.xi = dp + (size_t)total * n;
    S.t = dp + (size_t)total * 2 * n;
    S.h = S.t + total;
    int *ip = reinterpret_cast<int *>(dp + st_doubles);
    S.succ = ip;
    S.steps = ip + total;
    S.rejects = ip + 2 * total;
    S.nits = ip + 3 * total;
    S.status = ip + 4 * total;
    S.escal = ip + 5 * total;
    double *tab64 = reinterpret_cast<double *>(coef_p);
    float *tab32 = mixed ? reinterpret_cast<float *>(coef_p + coef64) : nullptr;

    PrepArgs pa;
    pa.n = n;
    pa.T = T;
    pa.n_inst = n_inst;
    pa.n_params = s->n_params;
    pa.n_slots = n_slots;
    pa.slot_ptr = s->d_slot_ptr;
    pa.slot_term = s->d_slot_term;
    pa.slot_mult = s->d_slot_mult;
    pa.term_const = s->d_term_const;
    pa.map_ptr = s->d_map_ptr;
    pa.map_col = s->d_map_col;
    pa.map_val = s->d_map_val;
    pa.params = reinterpret_cast<const double *>(p_target);
    pa.out64 = tab64;
    pa.out32 = tab32;
    HIP_TRY(launch_prep(pa, st));
    double *tab64_start = nullptr;
    float *tab32_start = nullptr;
    if (param) {
        // the start instance's tables (one per instance with per_instance_start)
        // go after the n_inst target tables
        tab64_start = tab64 + (size_t)n_inst * n_slots * 2;
        tab32_start = tab32 ? tab32 + (size_t)n_inst * n_slots * 2 : nullptr;
        PrepArgs p0 = pa;
        p0.n_inst = pis ? n_inst : 1;
        p0.params = reinterpret_cast<const double *>(p_start);
        p0.out64 = tab64_start;
        p0.out32 = tab32_start;
        HIP_TRY(launch_prep(p0, st));
    }
    if (prof) HIP_TRY(hipEventRecord(c->ev[1], st));

    InitArgs ia;
    ia.n = n;
    ia.n_start = n_start;
    ia.total = total;
    ia.deg2 = s->deg2;
    ia.eqdeg = eqdeg_of(s);
    ia.start = reinterpret_cast<const double *>(start);
    ia.start_per_inst = pis ? 1 : 0;
    ia.h0 = o.h0;
    ia.s = S;
    ia.retrack = 0;
    HIP_TRY(launch_init(ia, st));
    if (prof) HIP_TRY(hipEventRecord(c->ev[2], st));

    const int lanes = choose_lanes_per_path(o, s);
    if (lanes < 0)
        return fail(HC_E_INVALID, "opts.lanes_per_path = %d does not fit this system (n = %d, %s tables)",
                    o.lanes_per_path, n, s->layout == HC_LAYOUT_TERMS ? "term-list" : "dense");
    if (param && lanes == 1)
        return fail(HC_E_UNSUPPORTED, "hc_track: parameter homotopies need lanes_per_path 0, 4 or 8 and n >= 2");
    const int tpi = choose_tracks_per_item(o, n_start, lanes);
    const int per_inst = (n_start + tpi - 1) / tpi;
    TrackArgs ta;
    ta.gamma = reinterpret_cast<const double *>(gamma);
    ta.deg2 = s->deg2;
    ta.n = n;
    ta.n_start = n_start;
    ta.items_per_inst = per_inst;
    ta.tracks_per_item = tpi;
    ta.n_items = per_inst * n_inst;
    ta.total = total;
    ta.h0 = o.h0;
    ta.h_min = o.h_min;
    ta.h_max = o.h_max;
    ta.beta_inc = o.beta_inc;
    ta.beta_dec = o.beta_dec;
    ta.pred_tol = o.pred_tol;
    ta.inf2 = o.inf_bound * o.inf_bound;
    ta.n_inc = o.n_inc;
    ta.max_newton = o.max_newton;
    ta.max_steps = o.max_steps;
    ta.s = S;
    ta.n_suspended = reinterpret_cast<unsigned *>(counter_p);
    ta.head = reinterpret_cast<unsigned *>(counter_p + 32);
    ta.vars = s->d_vars;
    ta.n_tslots = s->T;
    ta.sdeg = sdeg_of(s);
    ta.eqdeg = eqdeg_of(s);
    const int wpb = 4;

    // one pass = launches until no path is left suspended by steps_per_launch
    // few = true: a pass over a few paths (re-tracking after the crossing check,
    // the end-game), which the one-path-per-wavefront tracker runs at a shorter
    // stage latency where it holds the system
    auto run_pass = [&](bool fp32, double t_final, int escalate, bool few) -> hc_status {
        const bool wave = !fp32 && wave_fits(s) && (few || lanes == 64);
        ta.coef = fp32 ? (const void *)tab32 : (const void *)tab64;
        ta.coef0 = !param ? nullptr : fp32 ? (const void *)tab32_start : (const void *)tab64_start;
        ta.coef0_stride = (param && pis) ? (long long)n_slots * 2 : 0;
        ta.coef64 = tab64;
        ta.coef0_64 = tab64_start;
        ta.tau = fp32 ? o.tau32 : o.tau64;
        ta.tau64 = o.tau64;
        ta.t_final = t_final;
        ta.t_switch = fp32 ? std::min(1.0 - o.t_end, t_final) : t_final;
        ta.escalate = escalate;
        ta.ir = fp32 && o.fp64_residual ? 1 : 0;
        ta.launch_steps = o.steps_per_launch;
        // the lane tracker sums into one counter, the group and wave trackers into
        // [FP32, FP64]
        ta.stage_count = !prof ? nullptr : (lanes == 1 && !wave) ? stage_ctr + (fp32 ? 0 : 1) : stage_ctr;
        for (;;) {
            if (o.steps_per_launch > 0) HIP_TRY(hipMemsetAsync(ta.n_suspended, 0, sizeof(unsigned), st));
            if (wave) {
                HIP_TRY(launch_track_wave(n, ta, reinterpret_cast<int *>(state_p + wave_off),
                                          reinterpret_cast<unsigned *>(counter_p + 56),
                                          (int)std::min<long long>(total, 4096), st));
            } else if (lanes == 1) {
                HIP_TRY(launch_track(n, fp32, ta, wpb, st));
            } else {
                HIP_TRY(launch_fill_u32(ta.head, 0u, 1, st));
                if (s->layout == HC_LAYOUT_TERMS) HIP_TRY(launch_track_terms(s->tk, fp32, ta, st));
                else HIP_TRY(launch_track_group(n, fp32, ta, st));
            }
            if (fp32) c->launches_fp32++;
            else c->launches_fp64++;
            if (o.steps_per_launch == 0) break;
            unsigned left = 0;
            HIP_TRY(hipMemcpyAsync(&left, ta.n_suspended, sizeof left, hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            if (left == 0) break;
        }
        return HC_OK;
    };
    if (lanes > 1 && mixed && inline_escalation(s)) {
        // group tracker: one launch; failed paths and the end zone go on in FP64
        // inside the kernel
        rc = run_pass(true, 1.0, 0, false);
        if (rc != HC_OK) return rc;
        c->had_fp32 = true;
        if (prof) HIP_TRY(hipEventRecord(c->ev[3], st));
    } else {
        // an FP32 pass to 1 - t_end that hands its failures back, then the FP64
        // pass
        if (mixed) {
            rc = run_pass(true, 1.0 - o.t_end, 1, false);
            if (rc != HC_OK) return rc;
            c->had_fp32 = true;
        }
        if (prof) HIP_TRY(hipEventRecord(c->ev[3], st));
        rc = run_pass(false, 1.0, 0, false);
        if (rc != HC_OK) return rc;
    }
    if (prof) HIP_TRY(hipEventRecord(c->ev[4], st));

    RefineArgs ra{};
    ra.coef = tab64;
    ra.gamma = reinterpret_cast<const double *>(gamma);
    ra.deg2 = s->deg2;
    ra.n_start = n_start;
    ra.total = total;
    ra.max_refine = o.max_refine;
    ra.tau_refine = o.tau_refine;
    ra.inf2 = o.inf_bound * o.inf_bound;
    ra.eta_max = o.eta_max;
    ra.s = S;
    ra.endpoints = reinterpret_cast<double *>(endpoints);
    ra.status = status;
    ra.info = info;
    ra.n = n;
    ra.n_tslots = s->T;
    ra.vars = s->d_vars;
    ra.sdeg = sdeg_of(s);
    if (s->layout == HC_LAYOUT_TERMS) HIP_TRY(launch_refine_terms(s->tk, ra, st));
    else HIP_TRY(launch_refine(n, ra, st));
    if (prof) HIP_TRY(hipEventRecord(c->ev[5], st));
    if (mixed && o.crossing_check) {
        // crossing check: paths that ended on the same root start over in FP64
        DedupArgs da;
        da.n = n;
        da.n_start = n_start;
        da.n_inst = n_inst;
        da.total = total;
        da.tol = kCrossTol;
        da.endpoints = reinterpret_cast<const double *>(endpoints);
        da.status = status;
        da.s = S;
        da.proj = big_check ? reinterpret_cast<double *>(state_p + proj_off) : nullptr;
        HIP_TRY(launch_dedup(da, st));
        InitArgs ir = ia;
        ir.retrack = 1;
        HIP_TRY(launch_init(ir, st));
        rc = run_pass(false, 1.0, 0, true);
        if (rc != HC_OK) return rc;
        if (s->layout == HC_LAYOUT_TERMS) HIP_TRY(launch_refine_terms(s->tk, ra, st));
        else HIP_TRY(launch_refine(n, ra, st));
    }
    if (o.endgame) {
        rc = run_endgame(c, s, o, total, S, ia, ra, counter_p, run_pass, ta, st);
        if (rc != HC_OK) return rc;
    }
    if (prof) {
        HIP_TRY(hipEventRecord(c->ev[6], st));
        c->profiled_call = true;
    }
    return HC_OK;
}

extern "C" {

hc_status hc_solve_batched_device(hc_ctx *c, int32_t n, int64_t batch, int32_t fp32, const void *A, const void *b,
                                  void *x, int32_t *info, void *stream)
{
    clear_error();
    if (!c) return fail(HC_E_INVALID, "hc_solve_batched_device: NULL context");
    if (n < 1 || n > 32) return fail(HC_E_INVALID, "hc_solve_batched_device: n = %d outside 1..32", n);
    if (batch < 0) return fail(HC_E_INVALID, "hc_solve_batched_device: batch = %lld", (long long)batch);
    if (batch == 0) return HC_OK;
    if (!A || !b || !x) return fail(HC_E_INVALID, "hc_solve_batched_device: NULL array");
    HIP_TRY(hipSetDevice(c->device));
    HIP_TRY(launch_lu_solve(n, batch, fp32 != 0, A, b, x, info, static_cast<hipStream_t>(stream)));
    return HC_OK;
}

hc_status hc_distinct_device(hc_ctx *c, int32_t n, int64_t count, const hc_c64 *points, double tol, int32_t *keep,
                             void *stream)
{
    clear_error();
    if (!c) return fail(HC_E_INVALID, "hc_distinct_device: NULL context");
    if (n < 1 || n > 64 || count < 0 || !(tol >= 0))
        return fail(HC_E_INVALID, "hc_distinct_device: n = %d (1..64), count = %lld, tol = %g", n, (long long)count,
                    tol);
    if (count == 0) return HC_OK;
    if (!points || !keep) return fail(HC_E_INVALID, "hc_distinct_device: NULL array");
    HIP_TRY(hipSetDevice(c->device));
    HIP_TRY(launch_distinct(n, count, reinterpret_cast<const double *>(points), tol, keep,
                            static_cast<hipStream_t>(stream)));
    return HC_OK;
}

hc_status hc_eval_dense_device(hc_ctx *c, const hc_system *s, const hc_c64 *p_target, int32_t n_inst,
                               const float *x, int32_t n_pts, int32_t engine, int32_t repeat, float *F, float *J,
                               void *stream)
{
    clear_error();
    if (!c || !s) return fail(HC_E_INVALID, "hc_eval_dense_device: NULL context or system");
    if (n_inst < 0 || n_pts < 0 || n_pts > (1 << 30) || repeat < 1 ||
        (engine != HC_EVAL_ROWS && engine != HC_EVAL_MFMA))
        return fail(HC_E_INVALID, "hc_eval_dense_device: n_inst = %d, n_pts = %d, repeat = %d, engine = %d", n_inst,
                    n_pts, repeat, engine);
    if (s->layout != HC_LAYOUT_DENSE || s->n > 8)
        return fail(HC_E_UNSUPPORTED, "hc_eval_dense_device: needs a dense-table system with n <= 8 (n = %d)", s->n);
    if ((long long)n_inst * n_pts == 0) return HC_OK;
    if (!x || !F || !J || (!p_target && s->n_params > 0))
        return fail(HC_E_INVALID, "hc_eval_dense_device: NULL array");
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int n_slots = s->n * s->T;
    const size_t b64 = (size_t)n_inst * n_slots * 2 * sizeof(double);
    HIP_TRY(c->evtab.ensure(b64 + (size_t)n_inst * n_slots * 2 * sizeof(float)));
    PrepArgs pa;
    pa.n = s->n;
    pa.T = s->T;
    pa.n_inst = n_inst;
    pa.n_params = s->n_params;
    pa.n_slots = n_slots;
    pa.slot_ptr = s->d_slot_ptr;
    pa.slot_term = s->d_slot_term;
    pa.slot_mult = s->d_slot_mult;
    pa.term_const = s->d_term_const;
    pa.map_ptr = s->d_map_ptr;
    pa.map_col = s->d_map_col;
    pa.map_val = s->d_map_val;
    pa.params = reinterpret_cast<const double *>(p_target);
    pa.out64 = static_cast<double *>(c->evtab.p);
    pa.out32 = reinterpret_cast<float *>(static_cast<char *>(c->evtab.p) + b64);
    HIP_TRY(launch_prep(pa, st));
    EvalArgs ea;
    ea.n = s->n;
    ea.n_inst = n_inst;
    ea.n_pts = n_pts;
    ea.repeat = repeat;
    ea.tab = pa.out32;
    ea.x = x;
    ea.F = F;
    ea.J = J;
    HIP_TRY(launch_eval(ea, engine, st));
    return HC_OK;
}

hc_status hc_measure_vector_peak(hc_ctx *c, int32_t fp64, double *tflops)
{
    clear_error();
    if (!c || !tflops) return fail(HC_E_INVALID, "hc_measure_vector_peak: NULL argument");
    HIP_TRY(hipSetDevice(c->device));
    double v = 0.0;
    HIP_TRY(measure_peak_fma(fp64 != 0, &v, nullptr));
    *tflops = v;
    return HC_OK;
}

hc_status hc_track_device(hc_ctx *c, const hc_system *s, const hc_c64 *start, int32_t n_start,
                          const hc_c64 *p_start, const hc_c64 *p_target, int32_t n_inst,
                          const hc_c64 *gamma, const hc_opts *opts, hc_c64 *endpoints, int32_t *status,
                          hc_track_info *info, void *stream)
{
    clear_error();
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool graph = c && opts && opts->use_graph && st != nullptr && opts->steps_per_launch == 0 &&
                       opts->endgame == 0 && !c->profiling;
    auto run = [&]() {
        return track_device_impl(c, s, start, n_start, p_start, p_target, n_inst, gamma, opts, endpoints, status,
                                 info, st);
    };
    if (!graph) return run();
    auto key = [&]() {
        std::vector<unsigned char> k;
        put(k, s);
        put(k, start);
        put(k, n_start);
        put(k, p_start);
        put(k, p_target);
        put(k, n_inst);
        put(k, gamma);
        put(k, *opts);
        put(k, endpoints);
        put(k, status);
        put(k, info);
        put(k, st);
        put(k, c->state.moves);
        put(k, c->coef.moves);
        put(k, c->counter.moves);
        return k;
    };
    if (c->graph_valid && key() == c->graph_key) {
        HIP_TRY(hipGraphLaunch(c->graph_exec, st));
        return HC_OK;
    }
    // First call with these arguments: run it (this also sizes the workspace),
    // then record the same launch sequence for replays.
    hc_status rc = run();
    if (rc != HC_OK) return rc;
    c->graph_valid = false;
    HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    rc = run();
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &g);
    if (rc != HC_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(HC_E_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    if (c->graph_exec) {
        (void)hipGraphExecDestroy(c->graph_exec);
        c->graph_exec = nullptr;
    }
    const hipError_t ei = hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return fail(HC_E_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(ei));
    c->graph_key = key();
    c->graph_valid = true;
    return HC_OK;
}

hc_status hc_track_device_noalloc(hc_ctx *c, const hc_system *s, const hc_c64 *start, int32_t n_start,
                                  const hc_c64 *p_start, const hc_c64 *p_target, int32_t n_inst,
                                  const hc_c64 *gamma, const hc_opts *opts, hc_c64 *endpoints, int32_t *status,
                                  hc_track_info *info, void *stream)
{
    clear_error();
    return track_device_impl(c, s, start, n_start, p_start, p_target, n_inst, gamma, opts, endpoints, status, info,
                             static_cast<hipStream_t>(stream), true);
}

hc_status hc_autotune(hc_ctx *c, const hc_system *s, const hc_c64 *start, int32_t n_start, const hc_c64 *p_start,
                      const hc_c64 *p_target, int32_t n_inst, const hc_c64 *gamma, const hc_opts *opts,
                      hc_c64 *endpoints, int32_t *status, hc_track_info *info, void *stream, hc_opts *best)
{
    clear_error();
    if (!c || !s || !best) return fail(HC_E_INVALID, "hc_autotune: NULL argument");
    hc_opts o;
    if (opts) o = *opts;
    else hc_default_opts(&o);
    hc_status rc = check_opts(o);
    if (rc != HC_OK) return rc;
    const bool tune_spl = o.steps_per_launch < 0;
    o.use_graph = 0;
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_TRY(hipSetDevice(c->device));
    // candidates: table layout (the system's, and the other one where it can hold
    // the system) x lanes per path x paths per work item (x steps per launch
    // when asked for)
    struct Cand {
        const hc_system *sys;
        TuneChoice ch;
    };
    std::vector<Cand> cand;
    const hc_system *layouts[2] = {s, alt_layout(c, s)};
    for (const hc_system *ls : layouts) {
        if (!ls) continue;
        std::vector<std::pair<int, int>> lt;  // (lanes, paths per item)
        if (ls->n >= 2) {
            const int g = lanes_for(ls);
            for (int per_group : {1, 2, 4}) lt.push_back({g, per_group * (64 / g)});
        }
        if (ls->kind == HC_TOTAL_DEGREE && ls->layout == HC_LAYOUT_DENSE)
            for (int tpi : {64, 256}) lt.push_back({1, tpi});
        for (auto &x : lt)
            for (int spl : {0, 64, 512}) {
                if (spl && !tune_spl) continue;
                Cand cd;
                cd.sys = ls;
                cd.ch.layout = ls->layout;
                cd.ch.lanes = x.first;
                cd.ch.tpi = std::max(1, std::min(x.second, std::max(n_start, 1)));
                cd.ch.spl = spl;
                cand.push_back(cd);
            }
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best_ms = 0.0f;
    TuneChoice pick;
    for (const Cand &cd : cand) {
        hc_opts t = o;
        t.lanes_per_path = cd.ch.lanes;
        t.tracks_per_item = cd.ch.tpi;
        t.steps_per_launch = cd.ch.spl;
        t.table_layout = cd.ch.layout;
        rc = track_device_impl(c, s, start, n_start, p_start, p_target, n_inst, gamma, &t, endpoints, status,
                               info, st);
        if (rc != HC_OK) break;
        hipError_t e = hipEventRecord(e0, st);
        if (e == hipSuccess)
            rc = track_device_impl(c, s, start, n_start, p_start, p_target, n_inst, gamma, &t, endpoints,
                                   status, info, st);
        if (e == hipSuccess && rc == HC_OK) e = hipEventRecord(e1, st);
        if (e == hipSuccess && rc == HC_OK) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess && rc == HC_OK) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) rc = fail(HC_E_DEVICE, "hc_autotune: %s", hipGetErrorString(e));
        if (rc != HC_OK) break;
        if (pick.lanes == 0 || ms < best_ms) {
            best_ms = ms;
            pick = cd.ch;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != HC_OK) return rc;
    if (pick.lanes == 0) return fail(HC_E_UNSUPPORTED, "hc_autotune: no candidate applies to this system");
    c->tune[tune_key(c, s, o.precision, n_start, n_inst)] = pick;
    if (!c->tune_file.empty() && hc_tune_save(c, c->tune_file.c_str()) != HC_OK) return HC_E_INVALID;
    *best = o;
    if (opts) best->use_graph = opts->use_graph;
    best->lanes_per_path = pick.lanes;
    best->tracks_per_item = pick.tpi;
    best->steps_per_launch = pick.spl;
    best->table_layout = pick.layout;
    return HC_OK;
}

hc_status hc_tune_save(hc_ctx *c, const char *path)
{
    clear_error();
    if (!c || !path) return fail(HC_E_INVALID, "hc_tune_save: NULL argument");
    std::ofstream f(path, std::ios::trunc);
    if (!f) return fail(HC_E_INVALID, "hc_tune_save: cannot write %s", path);
    f << "# homotopy tracker autotuner cache: key -> layout lanes_per_path tracks_per_item steps_per_launch\n";
    for (const auto &e : c->tune)
        f << e.first << " -> " << e.second.layout << " " << e.second.lanes << " " << e.second.tpi << " "
          << e.second.spl << "\n";
    f.flush();
    if (!f) return fail(HC_E_INVALID, "hc_tune_save: write to %s failed", path);
    return HC_OK;
}

hc_status hc_tune_load(hc_ctx *c, const char *path, int32_t *n_loaded)
{
    clear_error();
    if (!c || !path) return fail(HC_E_INVALID, "hc_tune_load: NULL argument");
    std::ifstream f(path);
    if (!f) return fail(HC_E_INVALID, "hc_tune_load: cannot read %s", path);
    std::map<std::string, TuneChoice> got;
    std::string line;
    int lineno = 0;
    while (std::getline(f, line)) {
        lineno++;
        if (line.empty() || line[0] == '#') continue;
        const size_t arrow = line.find(" -> ");
        TuneChoice tc;
        if (arrow != std::string::npos) {
            std::istringstream v(line.substr(arrow + 4));
            if ((v >> tc.layout >> tc.lanes >> tc.tpi >> tc.spl) &&
                (tc.layout == HC_LAYOUT_DENSE || tc.layout == HC_LAYOUT_TERMS) && tc.lanes >= 1 && tc.tpi >= 1 &&
                tc.spl >= 0) {
                got[line.substr(0, arrow)] = tc;
                continue;
            }
        }
        return fail(HC_E_INVALID, "hc_tune_load: %s line %d is not 'key -> layout lanes tpi spl'", path, lineno);
    }
    for (auto &e : got) c->tune[e.first] = e.second;
    if (n_loaded) *n_loaded = (int32_t)got.size();
    return HC_OK;
}

hc_status hc_track(hc_ctx *c, const hc_system *s, const hc_c64 *start, int32_t n_start,
                   const hc_c64 *p_start, const hc_c64 *p_target, int32_t n_inst, const hc_c64 *gamma,
                   const hc_opts *opts, hc_c64 *endpoints, int32_t *status, hc_track_info *info)
{
    clear_error();
    if (!c || !s) return fail(HC_E_INVALID, "hc_track: NULL context or system");
    if (n_start < 0 || n_inst < 0) return fail(HC_E_INVALID, "hc_track: negative size");
    const long long total = (long long)n_start * n_inst;
    if (total == 0) return HC_OK;
    if (!endpoints || !status) return fail(HC_E_INVALID, "hc_track: NULL output");
    if (!p_target && s->n_params > 0) return fail(HC_E_INVALID, "hc_track: p_target is NULL");
    HIP_TRY(hipSetDevice(c->device));
    const int n = s->n;
    // device copies: start, p_target, gamma, endpoints, status, info
    const size_t per = (opts && opts->per_instance_start) ? (size_t)n_inst : 1;  // start sets
    const size_t b_start = start ? per * n_start * n * sizeof(hc_c64) : 0;
    const size_t b_par = (size_t)n_inst * s->n_params * sizeof(hc_c64);
    const size_t b_gam = gamma ? (size_t)n_inst * sizeof(hc_c64) : 0;
    const size_t b_p0 = p_start ? per * s->n_params * sizeof(hc_c64) : 0;
    const size_t b_ep = (size_t)total * n * sizeof(hc_c64);
    const size_t b_st = (size_t)total * sizeof(int32_t);
    const size_t b_inf = info ? (size_t)total * sizeof(hc_track_info) : 0;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t need = al(b_start) + al(b_par) + al(b_gam) + al(b_p0) + al(b_ep) + al(b_st) + al(b_inf);
    HIP_TRY(c->io.ensure(need));
    char *base = static_cast<char *>(c->io.p);
    size_t off = 0;
    auto take = [&](size_t b) -> void * {
        if (b == 0) return nullptr;
        void *p = base + off;
        off += al(b);
        return p;
    };
    hc_c64 *d_start = static_cast<hc_c64 *>(take(b_start));
    hc_c64 *d_par = static_cast<hc_c64 *>(take(b_par));
    hc_c64 *d_gam = static_cast<hc_c64 *>(take(b_gam));
    hc_c64 *d_p0 = static_cast<hc_c64 *>(take(b_p0));
    hc_c64 *d_ep = static_cast<hc_c64 *>(take(b_ep));
    int32_t *d_st = static_cast<int32_t *>(take(b_st));
    hc_track_info *d_inf = static_cast<hc_track_info *>(take(b_inf));
    hipStream_t st = c->own_stream;
    if (b_start) HIP_TRY(hipMemcpyAsync(d_start, start, b_start, hipMemcpyHostToDevice, st));
    if (b_par) HIP_TRY(hipMemcpyAsync(d_par, p_target, b_par, hipMemcpyHostToDevice, st));
    if (b_gam) HIP_TRY(hipMemcpyAsync(d_gam, gamma, b_gam, hipMemcpyHostToDevice, st));
    if (b_p0) HIP_TRY(hipMemcpyAsync(d_p0, p_start, b_p0, hipMemcpyHostToDevice, st));
    hc_status rc = track_device_impl(c, s, d_start, n_start, d_p0, d_par, n_inst, d_gam, opts, d_ep, d_st,
                                     d_inf, st);
    if (rc != HC_OK) {
        (void)hipStreamSynchronize(st);
        return rc;
    }
    HIP_TRY(hipMemcpyAsync(endpoints, d_ep, b_ep, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(status, d_st, b_st, hipMemcpyDeviceToHost, st));
    if (b_inf) HIP_TRY(hipMemcpyAsync(info, d_inf, b_inf, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return HC_OK;
}

}  // extern "C"

// The batch launch sequence.  upload = false (graph capture): the job blob is
// already on the device from the eager call with the same arguments, so only
// the kernels are enqueued.
static hc_status track_batch_impl(hc_ctx *c, int32_t n_jobs, const hc_job *jobs, const hc_opts &o, hipStream_t st,
                                  bool upload)
{
    hc_status rc = HC_OK;
    const bool mixed = o.precision == HC_MIXED;

    // per-job sizes and workspace offsets
    struct Plan {
        const hc_job *j;
        const hc_system *s;
        long long total;
        int n, T, n_slots, n_tab, tpi;
        bool param;
        size_t st_off, proj_off, tab64_off, tab32_off;
        InitArgs init;
    };
    std::vector<Plan> plan;
    size_t st_bytes = 0, tab_bytes = 0;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    for (int k = 0; k < n_jobs; k++) {
        const hc_job &j = jobs[k];
        if (!j.sys) return fail(HC_E_INVALID, "hc_track_batch_device: job %d has no system", k);
        const hc_system *s = j.sys;
        if (s->device != c->device)
            return fail(HC_E_INVALID, "hc_track_batch_device: job %d's system lives on another device", k);
        if (j.n_start < 0 || j.n_inst < 0) return fail(HC_E_INVALID, "hc_track_batch_device: job %d negative size", k);
        if (s->n < 2) return fail(HC_E_UNSUPPORTED, "hc_track_batch_device: job %d has n = 1", k);
        Plan p{};
        p.j = &j;
        p.s = s;
        p.n = s->n;
        p.T = s->T;
        p.n_slots = s->n * s->T;
        p.param = s->kind == HC_PARAMETER;
        p.total = (long long)j.n_start * j.n_inst;
        if (p.total > 0) {
            if (!p.param && !j.start && j.n_start > s->bezout)
                return fail(HC_E_INVALID, "hc_track_batch_device: job %d n_start exceeds the Bezout number", k);
            if (p.param && (!j.start || (!j.p_start && s->n_params > 0)))
                return fail(HC_E_INVALID, "hc_track_batch_device: job %d needs start points and p_start", k);
            if (!j.endpoints || !j.status || (!j.p_target && s->n_params > 0))
                return fail(HC_E_INVALID, "hc_track_batch_device: job %d has a NULL buffer", k);
        }
        p.n_tab = j.n_inst + (p.param ? 1 : 0);
        p.tpi = choose_tracks_per_item(o, j.n_start, lanes_for(s));
        p.st_off = st_bytes;
        st_bytes += al((size_t)p.total * ((2 * p.n + 2) * 8 + 6 * 4));
        p.proj_off = st_bytes;
        if (mixed_check_big(o, j.n_start)) st_bytes += al((size_t)p.total * 16);
        p.tab64_off = tab_bytes;
        tab_bytes += al((size_t)p.n_tab * p.n_slots * 16);
        p.tab32_off = tab_bytes;
        if (mixed) tab_bytes += al((size_t)p.n_tab * p.n_slots * 8);
        plan.push_back(p);
    }
    HIP_TRY(hipSetDevice(c->device));
    HIP_TRY(c->state.ensure(st_bytes));
    HIP_TRY(c->coef.ensure(tab_bytes));
    HIP_TRY(c->counter.ensure(64));
    unsigned long long *stage_ctr = reinterpret_cast<unsigned long long *>(static_cast<char *>(c->counter.p) + 16);

    // job descriptors (one set per pass) and the two queues (total degree, parameter)
    c->h_jobs.assign((size_t)2 * n_jobs, TrackArgs{});
    // per-job arguments of the steps around tracking, launched once for all jobs
    std::vector<PrepArgs> preps;
    std::vector<InitArgs> inits;
    long long max_prep = 0, max_total = 0;
    // queues: [dense | term lists] x [total degree | parameter]
    std::vector<QueueItem> qs[kQueues];
    std::vector<int> job_n(n_jobs);
    for (int k = 0; k < n_jobs; k++) {
        Plan &p = plan[k];
        job_n[k] = p.n;
        char *sb = static_cast<char *>(c->state.p) + p.st_off;
        TrackState S;
        double *dp = reinterpret_cast<double *>(sb);
        S.xr = dp;
        S.xi = dp + (size_t)p.total * p.n;
        S.t = dp + (size_t)p.total * 2 * p.n;
        S.h = S.t + p.total;
        int *ip = reinterpret_cast<int *>(dp + (size_t)p.total * (2 * p.n + 2));
        S.succ = ip;
        S.steps = ip + p.total;
        S.rejects = ip + 2 * p.total;
        S.nits = ip + 3 * p.total;
        S.status = ip + 4 * p.total;
        S.escal = ip + 5 * p.total;
        double *t64 = reinterpret_cast<double *>(static_cast<char *>(c->coef.p) + p.tab64_off);
        float *t32 = mixed ? reinterpret_cast<float *>(static_cast<char *>(c->coef.p) + p.tab32_off) : nullptr;
        const double *t64s = p.param ? t64 + (size_t)p.j->n_inst * p.n_slots * 2 : nullptr;
        const float *t32s = (p.param && t32) ? t32 + (size_t)p.j->n_inst * p.n_slots * 2 : nullptr;
        if (p.total == 0) continue;

        PrepArgs pa;
        pa.n = p.n;
        pa.T = p.T;
        pa.n_inst = p.j->n_inst;
        pa.n_params = p.s->n_params;
        pa.n_slots = p.n_slots;
        pa.slot_ptr = p.s->d_slot_ptr;
        pa.slot_term = p.s->d_slot_term;
        pa.slot_mult = p.s->d_slot_mult;
        pa.term_const = p.s->d_term_const;
        pa.map_ptr = p.s->d_map_ptr;
        pa.map_col = p.s->d_map_col;
        pa.map_val = p.s->d_map_val;
        pa.params = reinterpret_cast<const double *>(p.j->p_target);
        pa.out64 = t64;
        pa.out32 = t32;
        preps.push_back(pa);
        max_prep = std::max(max_prep, (long long)pa.n_inst * pa.n_slots);
        if (p.param) {
            PrepArgs p0 = pa;
            p0.n_inst = 1;
            p0.params = reinterpret_cast<const double *>(p.j->p_start);
            p0.out64 = const_cast<double *>(t64s);
            p0.out32 = const_cast<float *>(t32s);
            preps.push_back(p0);
        }
        InitArgs ia;
        ia.n = p.n;
        ia.n_start = p.j->n_start;
        ia.total = p.total;
        ia.deg2 = p.s->deg2;
        ia.eqdeg = eqdeg_of(p.s);
        ia.start = reinterpret_cast<const double *>(p.j->start);
        ia.start_per_inst = 0;
        ia.h0 = o.h0;
        ia.s = S;
        ia.retrack = 0;
        inits.push_back(ia);
        max_total = std::max(max_total, p.total);
        p.init = ia;

        for (int pass = 0; pass < 2; pass++) {
            const bool fp32 = pass == 0;
            TrackArgs &ta = c->h_jobs[(size_t)pass * n_jobs + k];
            ta.n = p.n;
            ta.coef = fp32 ? (const void *)t32 : (const void *)t64;
            ta.coef0 = !p.param ? nullptr : fp32 ? (const void *)t32s : (const void *)t64s;
            ta.gamma = reinterpret_cast<const double *>(p.j->gamma);
            ta.deg2 = p.s->deg2;
            ta.n_start = p.j->n_start;
            ta.tracks_per_item = p.tpi;
            ta.items_per_inst = (p.j->n_start + p.tpi - 1) / p.tpi;
            ta.n_items = ta.items_per_inst * p.j->n_inst;
            ta.total = p.total;
            // in-kernel escalation: one launch in mixed mode, the FP32 tracker goes
            // on in FP64; otherwise an FP32 pass to 1 - t_end and an FP64 pass
            ta.coef64 = t64;
            ta.coef0_64 = t64s;
            ta.t_final = (fp32 && !kInlineEsc) ? 1.0 - o.t_end : 1.0;
            ta.t_switch = fp32 ? 1.0 - o.t_end : 1.0;
            ta.tau64 = o.tau64;
            ta.launch_steps = 0;
            ta.escalate = 0;
            ta.ir = fp32 && o.fp64_residual ? 1 : 0;
            ta.h0 = o.h0;
            ta.h_min = o.h_min;
            ta.h_max = o.h_max;
            ta.beta_inc = o.beta_inc;
            ta.beta_dec = o.beta_dec;
            ta.tau = fp32 ? o.tau32 : o.tau64;
            ta.pred_tol = o.pred_tol;
            ta.inf2 = o.inf_bound * o.inf_bound;
            ta.n_inc = o.n_inc;
            ta.max_newton = o.max_newton;
            ta.max_steps = o.max_steps;
            ta.s = S;
            ta.n_suspended = static_cast<unsigned *>(c->counter.p);
            ta.stage_count = c->profiling ? stage_ctr : nullptr;
            ta.vars = p.s->d_vars;
            ta.n_tslots = p.s->T;
            ta.sdeg = sdeg_of(p.s);
            ta.eqdeg = eqdeg_of(p.s);
        }
        std::vector<QueueItem> &q = qs[(p.s->layout == HC_LAYOUT_TERMS ? 2 + 2 * p.s->tk : 0) + (p.param ? 1 : 0)];
        for (int i = 0; i < p.j->n_inst; i++)
            for (int tb = 0; tb < p.j->n_start; tb += p.tpi)
                q.push_back({k, i, tb, std::min(tb + p.tpi, p.j->n_start)});
    }
    // larger systems first: their items are the longest
    auto by_n = [&](const QueueItem &x, const QueueItem &y) { return job_n[x.job] > job_n[y.job]; };
    c->h_items.clear();
    int q_off[kQueues + 1] = {};
    for (int qi = 0; qi < kQueues; qi++) {
        std::stable_sort(qs[qi].begin(), qs[qi].end(), by_n);
        c->h_items.insert(c->h_items.end(), qs[qi].begin(), qs[qi].end());
        q_off[qi + 1] = (int)c->h_items.size();
    }
    // refinement, crossing-check and re-tracking arguments per job; refinement
    // launches once per dense n and once for the term lists
    std::vector<RefineArgs> refs[kRefSlots];  // [n] dense, [kMaxN + 1 + kind] term lists
    std::vector<DedupArgs> dedups, big_dedups;  // big: instances above kDedupMax paths
    std::vector<InitArgs> retracks;
    long long ref_items[kRefSlots] = {}, ref_total[kRefSlots] = {};
    int max_inst = 0, max_start = 0;
    for (int k = 0; k < n_jobs; k++) {
        const Plan &p = plan[k];
        if (p.total == 0) continue;
        const TrackArgs &ta = c->h_jobs[(size_t)n_jobs + k];
        RefineArgs ra{};
        ra.coef = static_cast<const double *>(ta.coef);
        ra.gamma = ta.gamma;
        ra.deg2 = p.s->deg2;
        ra.n_start = p.j->n_start;
        ra.total = p.total;
        ra.max_refine = o.max_refine;
        ra.tau_refine = o.tau_refine;
        ra.inf2 = o.inf_bound * o.inf_bound;
        ra.eta_max = o.eta_max;
        ra.s = ta.s;
        ra.endpoints = reinterpret_cast<double *>(p.j->endpoints);
        ra.status = p.j->status;
        ra.info = p.j->info;
        ra.n = p.n;
        ra.n_tslots = p.s->T;
        ra.vars = p.s->d_vars;
        ra.sdeg = sdeg_of(p.s);
        const int rk = p.s->layout == HC_LAYOUT_TERMS ? kMaxN + 1 + p.s->tk : p.n;
        refs[rk].push_back(ra);
        ref_items[rk] = std::max(ref_items[rk], rk > kMaxN ? p.total
                                                                : (long long)p.j->n_inst * ((p.j->n_start + 63) / 64));
        ref_total[rk] = std::max(ref_total[rk], p.total);
        DedupArgs da;
        da.n = p.n;
        da.n_start = p.j->n_start;
        da.n_inst = p.j->n_inst;
        da.total = p.total;
        da.tol = kCrossTol;
        da.endpoints = reinterpret_cast<const double *>(p.j->endpoints);
        da.status = p.j->status;
        da.s = ta.s;
        da.proj = nullptr;
        if (mixed_check_big(o, p.j->n_start)) {
            da.proj = reinterpret_cast<double *>(static_cast<char *>(c->state.p) + p.proj_off);
            big_dedups.push_back(da);
        }
        dedups.push_back(da);
        max_inst = std::max(max_inst, p.j->n_inst);
        max_start = std::max(max_start, p.j->n_start);
        InitArgs ir = p.init;
        ir.retrack = 1;
        retracks.push_back(ir);
    }

    // one upload: job descriptors, work items, per-step argument arrays, queue heads
    size_t off = 0;
    auto place = [&](size_t bytes) {
        const size_t at = off;
        off += al(std::max<size_t>(bytes, 1));
        return at;
    };
    const size_t o_jobs = place(c->h_jobs.size() * sizeof(TrackArgs));
    const size_t o_items = place(c->h_items.size() * sizeof(QueueItem));
    const size_t o_prep = place(preps.size() * sizeof(PrepArgs));
    const size_t o_init = place(inits.size() * sizeof(InitArgs));
    const size_t o_dedup = place(dedups.size() * sizeof(DedupArgs));
    const size_t o_retr = place(retracks.size() * sizeof(InitArgs));
    size_t o_ref[kRefSlots];
    for (int rk = 0; rk < kRefSlots; rk++) o_ref[rk] = place(refs[rk].size() * sizeof(RefineArgs));
    const size_t o_heads = place(kQueues * sizeof(unsigned));
    c->h_blob.assign(off, 0);
    auto put_arr = [&](size_t at, const void *src, size_t bytes) {
        if (bytes) std::memcpy(c->h_blob.data() + at, src, bytes);
    };
    put_arr(o_jobs, c->h_jobs.data(), c->h_jobs.size() * sizeof(TrackArgs));
    put_arr(o_items, c->h_items.data(), c->h_items.size() * sizeof(QueueItem));
    put_arr(o_prep, preps.data(), preps.size() * sizeof(PrepArgs));
    put_arr(o_init, inits.data(), inits.size() * sizeof(InitArgs));
    put_arr(o_dedup, dedups.data(), dedups.size() * sizeof(DedupArgs));
    put_arr(o_retr, retracks.data(), retracks.size() * sizeof(InitArgs));
    for (int rk = 0; rk < kRefSlots; rk++) put_arr(o_ref[rk], refs[rk].data(), refs[rk].size() * sizeof(RefineArgs));
    HIP_TRY(c->queue.ensure(off));
    char *qb = static_cast<char *>(c->queue.p);
    if (upload) HIP_TRY(hipMemcpyAsync(qb, c->h_blob.data(), o_heads, hipMemcpyHostToDevice, st));
    TrackArgs *d_jobs = reinterpret_cast<TrackArgs *>(qb + o_jobs);
    QueueItem *d_items = reinterpret_cast<QueueItem *>(qb + o_items);
    unsigned *heads = reinterpret_cast<unsigned *>(qb + o_heads);

    HIP_TRY(launch_prep_many(reinterpret_cast<const PrepArgs *>(qb + o_prep), (int)preps.size(), max_prep, st));
    HIP_TRY(launch_init_many(reinterpret_cast<const InitArgs *>(qb + o_init), (int)inits.size(), max_total, st));
    auto run_pass = [&](bool fp32) -> hc_status {
        const TrackArgs *pj = d_jobs + (fp32 ? 0 : n_jobs);
        HIP_TRY(launch_fill_u32(heads, 0u, kQueues, st));
        for (int qi = 0; qi < kQueues; qi++) {
            const int cnt = q_off[qi + 1] - q_off[qi];
            if (cnt == 0) continue;
            const bool param = (qi & 1) != 0;
            if (qi < 2)
                HIP_TRY(launch_track_queue(fp32, param, pj, d_items + q_off[qi], cnt, heads + qi,
                                           queue_waves(fp32, param), st));
            else
                HIP_TRY(launch_track_queue_terms((qi - 2) / 2, fp32, param, pj, d_items + q_off[qi], cnt, heads + qi,
                                                 queue_waves_terms((qi - 2) / 2, fp32, param), st));
        }
        return HC_OK;
    };
    auto refine_all = [&]() -> hc_status {
        for (int rk = 1; rk < kRefSlots; rk++) {
            if (refs[rk].empty()) continue;
            const RefineArgs *d = reinterpret_cast<const RefineArgs *>(qb + o_ref[rk]);
            if (rk > kMaxN)
                HIP_TRY(launch_refine_terms_many(rk - kMaxN - 1, d, (int)refs[rk].size(), ref_items[rk], st));
            else
                HIP_TRY(launch_refine_many(rk, d, (int)refs[rk].size(), ref_items[rk], ref_total[rk], st));
        }
        return HC_OK;
    };
    rc = run_pass(mixed);
    if (rc != HC_OK) return rc;
    // the batch tracker escalates inline on every kind (k_track_queue_terms)
    if (mixed && !kInlineEsc) {
        rc = run_pass(false);
        if (rc != HC_OK) return rc;
    }
    rc = refine_all();
    if (rc != HC_OK) return rc;
    if (mixed && o.crossing_check) {
        // crossing check of every job, one FP64 pass over the queues, then the
        // refinement of the re-tracked paths
        HIP_TRY(launch_dedup_many(reinterpret_cast<const DedupArgs *>(qb + o_dedup), (int)dedups.size(), max_inst,
                                  max_start, st));
        for (const DedupArgs &da : big_dedups) HIP_TRY(launch_dedup_big(da, st));
        HIP_TRY(launch_init_many(reinterpret_cast<const InitArgs *>(qb + o_retr), (int)retracks.size(), max_total,
                                 st));
        rc = run_pass(false);
        if (rc != HC_OK) return rc;
        rc = refine_all();
        if (rc != HC_OK) return rc;
    }
    return HC_OK;
}

extern "C" {

hc_status hc_track_batch_device(hc_ctx *c, int32_t n_jobs, const hc_job *jobs, const hc_opts *opts_in,
                                void *stream)
{
    clear_error();
    if (!c || n_jobs < 0 || (n_jobs > 0 && !jobs)) return fail(HC_E_INVALID, "hc_track_batch_device: bad arguments");
    hc_opts o;
    if (opts_in) o = *opts_in;
    else hc_default_opts(&o);
    hc_status rc = check_opts(o);
    if (rc != HC_OK) return rc;
    if (o.steps_per_launch > 0 || o.lanes_per_path == 1)
        return fail(HC_E_UNSUPPORTED, "hc_track_batch_device: needs steps_per_launch 0 (or -1) and lanes_per_path "
                                      "0/4/8");
    o.steps_per_launch = 0;
    if (o.per_instance_start)
        return fail(HC_E_UNSUPPORTED, "hc_track_batch_device: per_instance_start is not available in a batch");
    if (o.endgame)
        return fail(HC_E_UNSUPPORTED, "hc_track_batch_device: the end-game is not available in a batch");
    if (o.table_layout != HC_LAYOUT_AUTO)
        return fail(HC_E_UNSUPPORTED, "hc_track_batch_device: table_layout must be 0 (each job's own)");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool graph = o.use_graph && st != nullptr && !c->profiling;
    if (!graph) return track_batch_impl(c, n_jobs, jobs, o, st, true);
    auto key = [&]() {
        std::vector<unsigned char> k;
        put(k, n_jobs);
        for (int j = 0; j < n_jobs; j++) put(k, jobs[j]);
        put(k, o);
        put(k, st);
        put(k, c->state.moves);
        put(k, c->coef.moves);
        put(k, c->counter.moves);
        put(k, c->queue.moves);
        return k;
    };
    if (c->bgraph_valid && key() == c->bgraph_key) {
        HIP_TRY(hipGraphLaunch(c->bgraph_exec, st));
        return HC_OK;
    }
    // first call with these arguments: run it eagerly (sizes the workspace and
    // uploads the job blob), then record its kernels for replays
    rc = track_batch_impl(c, n_jobs, jobs, o, st, true);
    if (rc != HC_OK) return rc;
    c->bgraph_valid = false;
    HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    rc = track_batch_impl(c, n_jobs, jobs, o, st, false);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &g);
    if (rc != HC_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(HC_E_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    if (c->bgraph_exec) {
        (void)hipGraphExecDestroy(c->bgraph_exec);
        c->bgraph_exec = nullptr;
    }
    const hipError_t ei = hipGraphInstantiate(&c->bgraph_exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return fail(HC_E_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(ei));
    c->bgraph_key = key();
    c->bgraph_valid = true;
    return HC_OK;
}

hc_status hc_set_profiling(hc_ctx *c, int32_t enable)
{
    clear_error();
    if (!c) return fail(HC_E_INVALID, "hc_set_profiling: NULL context");
    c->profiling = enable != 0;
    return HC_OK;
}

hc_status hc_last_profile(hc_ctx *c, hc_profile *out)
{
    clear_error();
    if (!c || !out) return fail(HC_E_INVALID, "hc_last_profile: NULL argument");
    if (!c->profiled_call) return fail(HC_E_INVALID, "hc_last_profile: no profiled call on this context");
    HIP_TRY(hipSetDevice(c->device));
    HIP_TRY(hipEventSynchronize(c->ev[6]));
    float ms[6];
    for (int i = 0; i < 6; i++) HIP_TRY(hipEventElapsedTime(&ms[i], c->ev[i], c->ev[i + 1]));
    unsigned long long cnt[2];
    HIP_TRY(hipMemcpy(cnt, static_cast<char *>(c->counter.p) + 16, sizeof cnt, hipMemcpyDeviceToHost));
    std::memset(out, 0, sizeof *out);
    out->ms_prep = ms[0];
    out->ms_init = ms[1];
    out->ms_track_fp32 = c->had_fp32 ? ms[2] : 0.0f;
    out->ms_track_fp64 = ms[3];
    out->ms_refine = ms[4];
    out->ms_crossing = ms[5];
    out->launches_fp32 = c->launches_fp32;
    out->launches_fp64 = c->launches_fp64;
    out->stages_fp32 = (int64_t)cnt[0];
    out->stages_fp64 = (int64_t)cnt[1];
    return HC_OK;
}

// Homogenised term tables (section 6): see hc.h.
hc_status hc_homogenize(int32_t n, int32_t n_entries, const int32_t *entry_ptr, const int32_t *scalar,
                        const int32_t *coef, const int32_t *exp, int32_t K, int32_t M, int32_t *out)
{
    clear_error();
    if (n < 1 || n_entries < 0 || K < 1 || M < 1)
        return fail(HC_E_INVALID, "hc_homogenize: bad sizes n=%d entries=%d K=%d M=%d", n, n_entries, K, M);
    if (n_entries > 0 && (!entry_ptr || !out)) return fail(HC_E_INVALID, "hc_homogenize: NULL argument");
    if (n_entries > 0 && entry_ptr[0] != 0) return fail(HC_E_INVALID, "hc_homogenize: entry_ptr[0] != 0");
    const int W = 2 + M;
    for (int e = 0; e < n_entries; e++) {
        const int t0 = entry_ptr[e], t1 = entry_ptr[e + 1];
        if (t1 < t0) return fail(HC_E_INVALID, "hc_homogenize: entry_ptr decreases at %d", e);
        if (t1 - t0 > K) return fail(HC_E_INVALID, "hc_homogenize: entry %d has %d terms > K = %d", e, t1 - t0, K);
        if (t1 > t0 && (!scalar || !coef || !exp)) return fail(HC_E_INVALID, "hc_homogenize: NULL term arrays");
        for (int t = t0; t < t1; t++) {
            int deg = 0;
            for (int j = 0; j < n; j++) {
                if (exp[(size_t)t * n + j] < 0) return fail(HC_E_INVALID, "hc_homogenize: negative exponent");
                deg += exp[(size_t)t * n + j];
            }
            if (deg > M) return fail(HC_E_INVALID, "hc_homogenize: term %d has degree %d > M = %d", t, deg, M);
        }
    }
    for (int e = 0; e < n_entries; e++) {
        const int t0 = entry_ptr[e], t1 = entry_ptr[e + 1];
        for (int k = 0; k < K; k++) {
            int32_t *row = out + ((size_t)e * K + k) * W;
            if (t0 + k < t1) {
                const int t = t0 + k;
                row[0] = scalar[t];
                row[1] = coef[t];
                int m = 0;
                for (int j = 0; j < n; j++)
                    for (int r = 0; r < exp[(size_t)t * n + j]; r++) row[2 + m++] = j;
                while (m < M) row[2 + m++] = n;  // auxiliary variable x_n = 1
            } else {
                // padding term: zero scalar, first coefficient, first variable
                for (int w = 0; w < W; w++) row[w] = 0;
            }
        }
    }
    return HC_OK;
}

}  // extern "C"
