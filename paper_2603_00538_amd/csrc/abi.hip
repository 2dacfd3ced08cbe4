// The extern "C" boundary: argument validation, call-order state, dispatch.
// No exception crosses it; every failure is a status plus ft_last_error().
#include <cmath>
#include <new>

#include "adaptive.h"
#include "common.h"

namespace ft {
const char* last_error();
ft_status target_setup(ft_target* T, const double* coords, const int32_t* conn, hipStream_t s);
ft_status solver_alloc(ft_target* T, hipStream_t s);
ft_status emit_points(ft_target* T, const ft_sample_cfg* cfg, void* points, hipStream_t s);
ft_status consume_values(ft_target* T, const ft_sample_cfg* cfg, const void* values, double* beta, hipStream_t s);
ft_status emit_points_varn(ft_target* T, const ft_sample_cfg* cfg, const int64_t* offs, int64_t total, void* points,
                           hipStream_t s);
ft_status consume_values_varn(ft_target* T, const ft_sample_cfg* cfg, const int64_t* offs, int64_t total,
                              const void* values, hipStream_t s);
size_t alloc_scratch_bytes(int64_t E);
ft_status allocate_samples(const double* var, int64_t E, int n0, int64_t budget, int n_min, int n_max,
                           int64_t* offs, void* scratch, int64_t* total, double* W, double* pred_var,
                           hipStream_t s);
ft_status project(ft_target* T, const ft_solve_cfg* cfg, double* x, double* b_out, ft_report* rep, hipStream_t s);
ft_status source_setup(ft_source* S, const double* coords, const int32_t* conn, const double* values,
                       const int32_t* bins, hipStream_t s);
ft_status source_eval(ft_source* S, int64_t head, int64_t npts, const void* pts, int64_t ld, int prec, void* out,
                      int64_t ld_out, int32_t* ids, hipStream_t s, unsigned long long* ood);
ft_status source_release(ft_source* S);
ft_status source_integral(ft_source* S, double* out, hipStream_t s);
ft_status source_eval_tiles(ft_source* S, int64_t n_nodes, int64_t n_elems, int N, const void* pts, int64_t ld,
                            int prec, void* out, int32_t* ids, hipStream_t s);
ft_status source_autotune(ft_source* S, int64_t head, int64_t npts, const void* pts, int64_t ld, int prec, int ncand,
                          const int32_t* cand, hipStream_t s);
ft_status transfer_p1(ft_target* T, ft_source* S, const ft_sample_cfg* cfg, hipStream_t s);
ft_status transfer_p1_varn(ft_target* T, ft_source* S, const ft_sample_cfg* cfg, const int64_t* offs, int64_t total,
                           hipStream_t s);
ft_status transfer_supermesh(ft_target* T, ft_source* S, double* area, hipStream_t s);
ft_status batch_setup(ft_batch* b, hipStream_t s);
ft_status batch_run(ft_batch* b, const ft_solve_cfg* cfg, double* const* x, double* const* bvec, ft_report* rep,
                    int32_t* status, hipStream_t s);
void batch_release(ft_batch* b);
ft_batch* batch_new(int count, ft_target* const* targets, ft_source* const* sources, const ft_sample_cfg* cfgs,
                    bool graph);
void batch_delete(ft_batch* b);
void batch_mark_consumed(ft_batch* b);
ft_status batch_autotune(ft_batch* b, const char* cache_path, int32_t* n_tuned, hipStream_t s);
void batch_variant(const ft_batch* b, int k, int32_t* G, int32_t* P);
int batch_count(const ft_batch* b);
ft_target* batch_target(const ft_batch* b, int k);
const ft_sample_cfg* batch_cfg(const ft_batch* b, int k);
bool batch_has_sources(const ft_batch* b);
ft_status batch_run_values(ft_batch* b, const ft_solve_cfg* cfg, const void* const* values, double* const* x,
                           double* const* bvec, ft_report* rep, int32_t* status, hipStream_t s);
ft_status plan_setup(ft_plan* pl, hipStream_t s);
ft_status plan_transfer(ft_plan* pl, const double* vals, hipStream_t s);
ft_plan* plan_new(ft_target* T, ft_source* S, const ft_sample_cfg* cfg);
void plan_delete(ft_plan* p);
ft_target* plan_target(ft_plan* p);
const ft_sample_cfg* plan_cfg(const ft_plan* p);
size_t noalloc_scratch_bytes();
ft_status noalloc_scratch(double** out);

static void target_release(ft_target* T) {
    void* ps[] = {T->coords, T->conn, T->vol, T->rowptr, T->col, T->val, T->diag, T->lumped, T->inc_ptr, T->inc,
                  T->beta, T->g, T->bres, T->r, T->z, T->p, T->q, T->y, T->b, T->scal, T->partials,
                  T->counters, T->val32, T->diag32, T->w32, T->scal32, T->mf_vec, T->mf_sc, T->mf_part,
                  T->var_el, T->var_tot, T->var_part};
    for (void* p : ps) dev_free(p);
    if (T->dofs != T->conn) dev_free(T->dofs);
    if (T->h_scal) (void)hipHostFree(T->h_scal);
    if (T->h_var) (void)hipHostFree(T->h_var);
}

ft_status check_sample_cfg(const ft_target* T, const ft_sample_cfg* cfg) {
    FT_ARG_CHECK(cfg, "cfg is null");
    FT_ARG_CHECK(cfg->samples_per_elem >= 1, "samples_per_elem must be >= 1 (got %d)", cfg->samples_per_elem);
    FT_ARG_CHECK(cfg->n_fields >= 1, "n_fields must be >= 1 (got %d)", cfg->n_fields);
    FT_ARG_CHECK(cfg->precision >= FT_F64 && cfg->precision <= FT_SPLIT_BF16, "precision out of range (%d)",
                 cfg->precision);
    FT_ARG_CHECK(std::isfinite(cfg->alpha), "alpha must be finite");
    FT_ARG_CHECK(cfg->sampling == FT_SAMPLING_PLAIN || cfg->sampling == FT_SAMPLING_STRATIFIED,
                 "sampling out of range (%d)", cfg->sampling);
    FT_ARG_CHECK(cfg->alpha_mode == FT_ALPHA_FIXED || cfg->alpha_mode == FT_ALPHA_ELEMENT,
                 "alpha_mode out of range (%d)", cfg->alpha_mode);
    FT_ARG_CHECK(cfg->values_layout == FT_VALUES_FIELD_MAJOR || cfg->values_layout == FT_VALUES_ELEMENT_TILES,
                 "values_layout out of range (%d)", cfg->values_layout);
    if (T->dim > 3 && (cfg->precision == FT_SPLIT_F16 || cfg->precision == FT_SPLIT_BF16)) {
        set_error("targets of dimension 4 to 6 take the FT_F64 and FT_F32 forms");
        return FT_E_UNSUPPORTED;
    }
    if (uint64_t(T->E) * uint64_t(cfg->samples_per_elem) >= (uint64_t(1) << 32) ||
        uint64_t(T->E) * 64u >= (uint64_t(1) << 32)) {
        set_error("n_elems * max(samples_per_elem, 64) must stay below 2^32 per transfer");
        return FT_E_UNSUPPORTED;
    }
    return FT_OK;
}

ft_status ensure_field_buffers(ft_target* T, int F, hipStream_t stream) {
    T->fields_inner = false;   // routes that keep the fields inner set it again
    if (F <= T->F_cap) return FT_OK;
    // buffers may still be read by queued work of an earlier transfer
    FT_TRY_HIP(hipStreamSynchronize(stream));
    dev_free(T->beta);
    dev_free(T->g);
    dev_free(T->bres);
    dev_free(T->var_el);
    dev_free(T->var_tot);
    dev_free(T->var_part);
    if (T->h_var) (void)hipHostFree(T->h_var);
    T->beta = T->g = T->bres = T->var_el = T->var_tot = T->var_part = T->h_var = nullptr;
    T->F_cap = 0;
    T->var_mode = VAR_NONE;
    FT_TRY(dev_alloc_n(&T->beta, size_t(F) * size_t(T->E) * T->nb));
    FT_TRY(dev_alloc_n(&T->g, size_t(F) * size_t(T->n)));
    FT_TRY(dev_alloc_n(&T->bres, size_t(F) * size_t(T->n)));
    FT_TRY(dev_alloc_n(&T->var_el, size_t(F) * size_t(T->E)));
    FT_TRY(dev_alloc_n(&T->var_tot, size_t(F)));
    FT_TRY(dev_alloc_n(&T->var_part, size_t(F) * kVarBlocks * 2));
    FT_TRY_HIP(hipHostMalloc((void**)&T->h_var, size_t(F) * sizeof(double), hipHostMallocDefault));
    T->F_cap = F;
    return FT_OK;
}

// binary32 point forms (FT_F32 and the split forms) sample the same points
static bool point_f32(int prec) { return prec != FT_F64; }

static bool same_samples(const ft_sample_cfg& a, const ft_sample_cfg& b) {
    return a.samples_per_elem == b.samples_per_elem && a.seed == b.seed && a.stream_id == b.stream_id &&
           a.sampling == b.sampling && point_f32(a.precision) == point_f32(b.precision);
}

// Each element's own control coefficient is computed by the black-box
// consumption kernel only (binary64 and binary32 forms, P1 targets).
static ft_status check_alpha_mode(const ft_target* T, const ft_sample_cfg* cfg, bool black_box) {
    if (cfg->alpha_mode == FT_ALPHA_ELEMENT &&
        (!black_box || cfg->precision == FT_SPLIT_F16 || cfg->precision == FT_SPLIT_BF16 || T->order != 1)) {
        set_error("per-element control coefficients are computed by ft_consume_queries in the FT_F64 and FT_F32 "
                  "forms on P1 targets only");
        return FT_E_UNSUPPORTED;
    }
    if (T->order != 1 && cfg->precision != FT_F64 && cfg->precision != FT_F32) {
        set_error("P2 targets take the FT_F64 and FT_F32 forms");
        return FT_E_UNSUPPORTED;
    }
    return FT_OK;
}

// What ft_project needs of the last consumption: with per-element
// coefficients the control part is inside the element loads (alpha = 0 there).
static ft_sample_cfg consumed_view(const ft_sample_cfg& c) {
    ft_sample_cfg v = c;
    if (c.alpha_mode == FT_ALPHA_ELEMENT) v.alpha = 0.0;
    return v;
}

}  // namespace ft

using namespace ft;

#define FT_GUARD_BEGIN try {
#define FT_GUARD_END                                  \
    }                                                 \
    catch (const std::bad_alloc&) {                   \
        set_error("host allocation failed");          \
        return FT_E_OOM;                              \
    }                                                 \
    catch (...) {                                     \
        set_error("unexpected internal exception");   \
        return FT_E_DEVICE;                           \
    }

struct ft_target_ext : ft_target {
    bool sampled = false;
    ft_sample_cfg sampled_cfg{};
    // the last sampling's per-element counts (null: samples_per_elem each)
    const int64_t* sampled_offs = nullptr;
    int64_t sampled_total = 0;
    // device scratch of ft_allocate_samples
    void* alloc_tmp = nullptr;
    size_t alloc_tmp_bytes = 0;
};

extern "C" {

static ft_status target_create(int32_t dim, int order, int64_t n_nodes, const double* coords, int64_t n_elems,
                               const int32_t* conn, hipStream_t stream, ft_target** out) {
    FT_ARG_CHECK(out, "out is null");
    *out = nullptr;
    FT_ARG_CHECK(dim >= 2 && dim <= (order == 1 ? 6 : 3), "dim must lie in [2, %d] (got %d)", order == 1 ? 6 : 3,
                 dim);
    FT_ARG_CHECK(coords && conn, "coords and conn must be device pointers");
    const int nb = order == 1 ? dim + 1 : (dim + 1) * (dim + 2) / 2;
    FT_ARG_CHECK(n_nodes >= nb && n_nodes < INT32_MAX, "n_nodes out of range (%lld)", (long long)n_nodes);
    FT_ARG_CHECK(n_elems >= 1 && n_elems * nb < INT32_MAX, "n_elems out of range (%lld)", (long long)n_elems);
    auto* T = new ft_target_ext();
    T->dim = dim;
    T->order = order;
    T->n = n_nodes;
    T->E = n_elems;
    ft_status st = target_setup(T, coords, conn, stream);
    if (st == FT_OK) st = solver_alloc(T, stream);
    // one field's transfer buffers up front, so that a first one-field
    // transfer needs no allocation (ft_consume_queries_noalloc relies on it)
    if (st == FT_OK) st = ensure_field_buffers(T, 1, stream);
    if (st == FT_OK && hipStreamSynchronize(stream) != hipSuccess) {
        set_error("stream synchronization failed after setup");
        st = FT_E_DEVICE;
    }
    if (st != FT_OK) {
        (void)hipStreamSynchronize(stream);
        target_release(T);
        delete T;
        return st;
    }
    *out = T;
    return FT_OK;
}

ft_status ft_target_create(int32_t dim, int64_t n_nodes, const double* coords, int64_t n_elems, const int32_t* conn,
                           hipStream_t stream, ft_target** out) {
    FT_GUARD_BEGIN
    clear_error();
    return target_create(dim, 1, n_nodes, coords, n_elems, conn, stream, out);
    FT_GUARD_END
}

ft_status ft_target_create_p2(int32_t dim, int64_t n_nodes, const double* coords, int64_t n_elems,
                              const int32_t* conn, hipStream_t stream, ft_target** out) {
    FT_GUARD_BEGIN
    clear_error();
    return target_create(dim, 2, n_nodes, coords, n_elems, conn, stream, out);
    FT_GUARD_END
}

ft_status ft_target_destroy(ft_target* t) {
    if (!t) return FT_OK;
    dev_free(static_cast<ft_target_ext*>(t)->alloc_tmp);
    target_release(t);
    delete static_cast<ft_target_ext*>(t);
    return FT_OK;
}

ft_status ft_target_get_info(const ft_target* t, ft_target_info* info) {
    clear_error();
    FT_ARG_CHECK(t && info, "null argument");
    info->dim = t->dim;
    info->n_nodes = t->n;
    info->n_elems = t->E;
    info->nnz = t->nnz;
    info->n_inverted = t->n_inverted;
    info->order = t->order;
    return FT_OK;
}

int64_t ft_query_count(const ft_target* t, int32_t samples_per_elem) {
    if (!t || samples_per_elem < 1) return -1;
    return t->n + t->E * int64_t(samples_per_elem);
}

ft_status ft_sample_points(ft_target* t, const ft_sample_cfg* cfg, void* points, hipStream_t stream) {
    FT_GUARD_BEGIN
    clear_error();
    FT_ARG_CHECK(t, "target is null");
    FT_TRY(check_sample_cfg(t, cfg));
    FT_ARG_CHECK(points, "points is null");
    FT_TRY(emit_points(t, cfg, points, stream));
    auto* T = static_cast<ft_target_ext*>(t);
    T->sampled = true;
    T->sampled_cfg = *cfg;
    T->sampled_offs = nullptr;
    return FT_OK;
    FT_GUARD_END
}

// Per-element counts: plain samples, field-major values, FT_F64 or FT_F32.
static ft_status check_varn_cfg(const ft_target* T, const ft_sample_cfg* cfg, const int64_t* offs, int64_t total) {
    FT_ARG_CHECK(cfg, "cfg is null");
    FT_ARG_CHECK(cfg->samples_per_elem == 0,
                 "samples_per_elem must be 0 when the counts come from offsets (got %d)", cfg->samples_per_elem);
    ft_sample_cfg c = *cfg;
    c.samples_per_elem = 1;
    FT_TRY(check_sample_cfg(T, &c));
    FT_ARG_CHECK(offs, "offsets is null");
    FT_ARG_CHECK(total >= T->E && total <= kMaxAllocTotal,
                 "total (%lld) must lie in [n_elems, 2^40]: every element takes at least one sample",
                 (long long)total);
    if (cfg->sampling != FT_SAMPLING_PLAIN || cfg->values_layout != FT_VALUES_FIELD_MAJOR ||
        (cfg->precision != FT_F64 && cfg->precision != FT_F32)) {
        set_error("per-element sample counts take plain samples, field-major values and the FT_F64 or FT_F32 form");
        return FT_E_UNSUPPORTED;
    }
    return FT_OK;
}

ft_status ft_allocate_samples(ft_target* t, int32_t field, int64_t budget, int32_t n_min, int32_t n_max,
                              int64_t* offsets, ft_allocation* out, hipStream_t stream) {
    FT_GUARD_BEGIN
    clear_error();
    FT_ARG_CHECK(t && offsets && out, "null argument");
    auto* T = static_cast<ft_target_ext*>(t);
    const int n0 = T->consumed_cfg.samples_per_elem;
    if (!T->consumed || T->var_mode != VAR_ESTIMATED || n0 < 2) {
        set_error("ft_allocate_samples needs a prior transfer with a fixed N >= 2 samples per element on a route "
                  "that estimates the element variances");
        return FT_E_ORDER;
    }
    FT_ARG_CHECK(field >= 0 && field < T->consumed_cfg.n_fields, "field %d out of range [0, %d)", field,
                 T->consumed_cfg.n_fields);
    FT_ARG_CHECK(n_min >= 1 && n_min <= n_max && n_max <= kMaxElemSamples,
                 "need 1 <= n_min <= n_max <= 2^20 (got %d, %d)", n_min, n_max);
    FT_ARG_CHECK(budget >= 1 && budget <= kMaxAllocTotal, "budget must lie in [1, 2^40] (got %lld)",
                 (long long)budget);
    // the counts add up to at most budget + n_elems / 2 before the clamps, which add at most n_elems * n_min
    FT_ARG_CHECK(double(budget) + double(T->E) * (double(n_min) + 1.0) <= double(kMaxAllocTotal),
                 "budget + n_elems * (n_min + 1) must stay within 2^40 samples");
    const size_t need = alloc_scratch_bytes(T->E);
    if (need > T->alloc_tmp_bytes) {
        FT_TRY_HIP(hipStreamSynchronize(stream));
        dev_free(T->alloc_tmp);
        T->alloc_tmp = nullptr;
        T->alloc_tmp_bytes = 0;
        FT_TRY(dev_alloc_n(reinterpret_cast<double**>(&T->alloc_tmp), need / sizeof(double)));
        T->alloc_tmp_bytes = need;
    }
    double W = 0.0, pv = 0.0;
    int64_t total = 0;
    FT_TRY(allocate_samples(T->var_el + int64_t(field) * T->E, T->E, n0, budget, n_min, n_max, offsets, T->alloc_tmp,
                            &total, &W, &pv, stream));
    out->total = total;
    out->weight_sum = W;
    out->predicted_stderr = std::sqrt(pv);
    return FT_OK;
    FT_GUARD_END
}

ft_status ft_sample_points_adaptive(ft_target* t, const ft_sample_cfg* cfg, const int64_t* offsets, int64_t total,
                                    void* points, hipStream_t stream) {
    FT_GUARD_BEGIN
    clear_error();
    FT_ARG_CHECK(t, "target is null");
    FT_TRY(check_varn_cfg(t, cfg, offsets, total));
    FT_ARG_CHECK(points, "points is null");
    FT_TRY(emit_points_varn(t, cfg, offsets, total, points, stream));
    auto* T = static_cast<ft_target_ext*>(t);
    T->sampled = true;
    T->sampled_cfg = *cfg;
    T->sampled_offs = offsets;
    T->sampled_total = total;
    return FT_OK;
    FT_GUARD_END
}

ft_status ft_consume_queries_adaptive(ft_target* t, const ft_sample_cfg* cfg, const int64_t* offsets, int64_t total,
                                      const void* values, hipStream_t stream) {
    FT_GUARD_BEGIN
    clear_error();
    FT_ARG_CHECK(t, "target is null");
    FT_TRY(check_varn_cfg(t, cfg, offsets, total));
    FT_ARG_CHECK(values, "values is null");
    auto* T = static_cast<ft_target_ext*>(t);
    if (!T->sampled || T->sampled_offs != offsets || T->sampled_total != total || !same_samples(T->sampled_cfg, *cfg)) {
        set_error("consume needs a prior ft_sample_points_adaptive with the same offsets, total, seed, stream_id "
                  "and point precision");
        return FT_E_ORDER;
    }
    FT_TRY(check_alpha_mode(T, cfg, true));
    FT_TRY(ensure_field_buffers(T, cfg->n_fields, stream));
    T->consumed = false;
    FT_TRY(consume_values_varn(T, cfg, offsets, total, values, stream));
    T->consumed = true;
    T->consumed_cfg = consumed_view(*cfg);
    return FT_OK;
    FT_GUARD_END
}

ft_status ft_consume_queries(ft_target* t, const ft_sample_cfg* cfg, const void* values, hipStream_t stream) {
    FT_GUARD_BEGIN
    clear_error();
    FT_ARG_CHECK(t, "target is null");
    FT_TRY(check_sample_cfg(t, cfg));
    FT_ARG_CHECK(values, "values is null");
    auto* T = static_cast<ft_target_ext*>(t);
    if (!T->sampled || !same_samples(T->sampled_cfg, *cfg)) {
        set_error("consume needs a prior ft_sample_points with the same samples_per_elem, seed, stream_id and "
                  "point precision");
        return FT_E_ORDER;
    }
    FT_TRY(check_alpha_mode(T, cfg, true));
    FT_TRY(ensure_field_buffers(T, cfg->n_fields, stream));
    T->consumed = false;
    FT_TRY(consume_values(T, cfg, values, T->beta, stream));
    T->consumed = true;
    T->consumed_cfg = consumed_view(*cfg);
    return FT_OK;
    FT_GUARD_END
}

ft_status ft_consume_queries_noalloc(ft_target* t, const ft_sample_cfg* cfg, const void* values,
                                     hipStream_t stream) {
    FT_GUARD_BEGIN
    clear_error();
    FT_ARG_CHECK(t, "target is null");
    FT_TRY(check_sample_cfg(t, cfg));
    FT_ARG_CHECK(values, "values is null");
    auto* T = static_cast<ft_target_ext*>(t);
    if (!T->sampled || !same_samples(T->sampled_cfg, *cfg)) {
        set_error("consume needs a prior ft_sample_points with the same samples_per_elem, seed, stream_id and "
                  "point precision");
        return FT_E_ORDER;
    }
    const uint64_t need = uint64_t(cfg->n_fields) * uint64_t(T->E) * uint64_t(T->nb) * sizeof(double);
    FT_ARG_CHECK(need <= noalloc_scratch_bytes(),
                 "the element loads of %d field(s) x %lld elements need %llu bytes; the scratch array holds %llu",
                 cfg->n_fields, (long long)T->E, (unsigned long long)need,
                 (unsigned long long)noalloc_scratch_bytes());
    FT_ARG_CHECK(cfg->n_fields <= T->F_cap,
                 "n_fields (%d) exceeds the %d field(s) the target holds buffers for (ft_consume_queries with "
                 "that field count provisions them)", cfg->n_fields, T->F_cap);
    FT_TRY(check_alpha_mode(T, cfg, true));
    double* scratch = nullptr;
    FT_TRY(noalloc_scratch(&scratch));
    T->fields_inner = false;   // the many-field route sets it again
    T->consumed = false;
    FT_TRY(consume_values(T, cfg, values, scratch, stream));
    T->consumed = true;
    T->consumed_cfg = consumed_view(*cfg);
    return FT_OK;
    FT_GUARD_END
}

ft_status ft_transfer_p1(ft_target* t, ft_source* s, const ft_sample_cfg* cfg, hipStream_t stream) {
    FT_GUARD_BEGIN
    clear_error();
    FT_ARG_CHECK(t && s, "target and source must be non-null");
    FT_TRY(check_sample_cfg(t, cfg));
    FT_ARG_CHECK(s->dim == t->dim, "source dimension %d differs from target dimension %d", s->dim, t->dim);
    FT_ARG_CHECK(cfg->n_fields == s->F, "n_fields (%d) must equal the source's field count (%d)", cfg->n_fields,
                 s->F);
    if ((cfg->precision != FT_F64 && cfg->precision != FT_F32) || cfg->n_fields > 4) {
        set_error("the fused built-in route supports FT_F64 and FT_F32 and at most 4 fields");
        return FT_E_UNSUPPORTED;
    }
    FT_TRY(check_alpha_mode(t, cfg, false));
    FT_TRY(ensure_field_buffers(t, cfg->n_fields, stream));
    t->consumed = false;
    FT_TRY(transfer_p1(t, s, cfg, stream));
    t->consumed = true;
    t->consumed_cfg = *cfg;
    return FT_OK;
    FT_GUARD_END
}

ft_status ft_transfer_p1_adaptive(ft_target* t, ft_source* s, const ft_sample_cfg* cfg, const int64_t* offsets,
                                  int64_t total, hipStream_t stream) {
    FT_GUARD_BEGIN
    clear_error();
    FT_ARG_CHECK(t && s, "target and source must be non-null");
    FT_TRY(check_varn_cfg(t, cfg, offsets, total));
    FT_ARG_CHECK(s->dim == t->dim, "source dimension %d differs from target dimension %d", s->dim, t->dim);
    FT_ARG_CHECK(cfg->n_fields == s->F, "n_fields (%d) must equal the source's field count (%d)", cfg->n_fields,
                 s->F);
    if (cfg->n_fields > 4) {
        set_error("the fused built-in route supports at most 4 fields");
        return FT_E_UNSUPPORTED;
    }
    FT_TRY(check_alpha_mode(t, cfg, false));
    FT_TRY(ensure_field_buffers(t, cfg->n_fields, stream));
    t->consumed = false;
    FT_TRY(transfer_p1_varn(t, s, cfg, offsets, total, stream));
    t->consumed = true;
    t->consumed_cfg = *cfg;
    return FT_OK;
    FT_GUARD_END
}

ft_status ft_transfer_supermesh(ft_target* t, ft_source* s, double* area, hipStream_t stream) {
    FT_GUARD_BEGIN
    clear_error();
    FT_ARG_CHECK(t && s, "target and source must be non-null");
    FT_ARG_CHECK(s->dim == t->dim, "source dimension %d differs from target dimension %d", s->dim, t->dim);
    if (s->F > 4 || t->order != 1) {
        set_error("the intersection route supports P1 targets and at most 4 fields");
        return FT_E_UNSUPPORTED;
    }
    FT_TRY(ensure_field_buffers(t, s->F, stream));
    t->consumed = false;
    FT_TRY(transfer_supermesh(t, s, area, stream));
    ft_sample_cfg c{};
    c.samples_per_elem = 0;
    c.n_fields = s->F;
    c.alpha = 0.0;   // exact load vector: no control part
    c.precision = FT_F64;
    t->consumed = true;
    t->consumed_cfg = c;
    return FT_OK;
    FT_GUARD_END
}

ft_status ft_project(ft_target* t, const ft_solve_cfg* cfg, double* x, double* b_out, ft_report* rep,
                     hipStream_t stream) {
    FT_GUARD_BEGIN
    clear_error();
    FT_ARG_CHECK(t && cfg && x && rep, "null argument");
    FT_ARG_CHECK(cfg->rtol >= 0.0 && std::isfinite(cfg->rtol), "rtol must be finite and >= 0");
    FT_ARG_CHECK(cfg->max_iter >= 0, "max_iter must be >= 0");
    FT_ARG_CHECK(cfg->refine_steps >= 0 && cfg->refine_steps <= 100, "refine_steps must lie in [0, 100]");
    if (!t->consumed) {
        set_error("ft_project needs a prior ft_consume_queries");
        return FT_E_ORDER;
    }
    return project(t, cfg, x, b_out, rep, stream);
    FT_GUARD_END
}

ft_status ft_plan_create(ft_target* t, ft_source* s, const ft_sample_cfg* cfg, hipStream_t stream, ft_plan** out) {
    FT_GUARD_BEGIN
    clear_error();
    FT_ARG_CHECK(out, "out is null");
    *out = nullptr;
    FT_ARG_CHECK(t && s, "target and source must be non-null");
    FT_TRY(check_sample_cfg(t, cfg));
    FT_ARG_CHECK(s->dim == t->dim, "source dimension %d differs from target dimension %d", s->dim, t->dim);
    FT_ARG_CHECK(cfg->n_fields == s->F, "n_fields (%d) must equal the source's field count (%d)", cfg->n_fields,
                 s->F);
    if (cfg->precision != FT_F64 || t->order != 1) {
        set_error("plans run the FT_F64 form on P1 targets");
        return FT_E_UNSUPPORTED;
    }
    FT_TRY(check_alpha_mode(t, cfg, false));
    FT_TRY(ensure_field_buffers(t, cfg->n_fields, stream));
    ft_plan* p = plan_new(t, s, cfg);
    const ft_status st = plan_setup(p, stream);
    if (st != FT_OK) {
        (void)hipStreamSynchronize(stream);
        plan_delete(p);
        return st;
    }
    *out = p;
    return FT_OK;
    FT_GUARD_END
}

ft_status ft_plan_transfer(ft_plan* p, const double* nodal_values, hipStream_t stream) {
    FT_GUARD_BEGIN
    clear_error();
    FT_ARG_CHECK(p, "plan is null");
    ft_target* t = plan_target(p);
    FT_TRY(ensure_field_buffers(t, plan_cfg(p)->n_fields, stream));
    t->consumed = false;
    FT_TRY(plan_transfer(p, nodal_values, stream));
    t->consumed = true;
    t->consumed_cfg = *plan_cfg(p);
    return FT_OK;
    FT_GUARD_END
}

ft_status ft_plan_destroy(ft_plan* p) {
    plan_delete(p);
    return FT_OK;
}

static bool sources_all_null(int count, ft_source* const* sources) {
    for (int k = 0; k < count; ++k)
        if (sources[k]) return false;
    return true;
}

ft_status ft_batch_create(int32_t count, ft_target* const* targets, ft_source* const* sources,
                          const ft_sample_cfg* cfgs, int32_t flags, hipStream_t stream, ft_batch** out) {
    FT_GUARD_BEGIN
    clear_error();
    FT_ARG_CHECK(out, "out is null");
    *out = nullptr;
    FT_ARG_CHECK(count >= 1 && count <= (1 << 20), "count out of range (%d)", count);
    FT_ARG_CHECK(targets && sources && cfgs, "targets, sources and cfgs must be host arrays");
    FT_ARG_CHECK((flags & ~FT_BATCH_GRAPH) == 0, "unknown flags 0x%x", flags);
    int64_t systems = 0;
    for (int k = 0; k < count; ++k) {
        const ft_target* t = targets[k];
        const ft_source* s = sources[k];
        FT_ARG_CHECK(t, "transfer %d: null target", k);
        if (t->dim > 3) {
            set_error("transfer %d: batches take triangle and tetrahedron targets", k);
            return FT_E_UNSUPPORTED;
        }
        FT_TRY(check_sample_cfg(t, &cfgs[k]));
        FT_ARG_CHECK(!s || s->dim == t->dim, "transfer %d: source dimension %d differs from target dimension %d", k,
                     s ? s->dim : 0, t->dim);
        FT_TRY(check_alpha_mode(t, &cfgs[k], false));
        FT_ARG_CHECK(!s || cfgs[k].n_fields == s->F,
                     "transfer %d: n_fields (%d) must equal the source's field count (%d)", k, cfgs[k].n_fields,
                     s ? s->F : 0);
        FT_ARG_CHECK(s || sources_all_null(count, sources), "transfer %d: either every transfer has a source or none",
                     k);
        if ((cfgs[k].precision != FT_F64 && cfgs[k].precision != FT_F32) || t->order != 1) {
            set_error("transfer %d: batches run FT_F64 or FT_F32 transfers to P1 targets", k);
            return FT_E_UNSUPPORTED;
        }
        systems += cfgs[k].n_fields;
        FT_ARG_CHECK(systems <= (1 << 20), "more than 2^20 fields in the batch");
        for (int j = 0; j < k; ++j)
            FT_ARG_CHECK(targets[j] != t, "transfers %d and %d share a target (its work buffers)", j, k);
    }
    ft_batch* b = batch_new(count, targets, sources, cfgs, (flags & FT_BATCH_GRAPH) != 0);
    const ft_status st = batch_setup(b, stream);
    if (st != FT_OK) {
        (void)hipStreamSynchronize(stream);
        batch_release(b);
        batch_delete(b);
        return st;
    }
    *out = b;
    return FT_OK;
    FT_GUARD_END
}

ft_status ft_batch_run(ft_batch* b, const ft_solve_cfg* cfg, double* const* x, double* const* bvec,
                       ft_report* reports, int32_t* status, hipStream_t stream) {
    FT_GUARD_BEGIN
    clear_error();
    FT_ARG_CHECK(b && cfg && x && reports, "null argument");
    FT_ARG_CHECK(cfg->rtol >= 0.0 && std::isfinite(cfg->rtol), "rtol must be finite and >= 0");
    FT_ARG_CHECK(cfg->max_iter >= 0 && cfg->max_iter <= 100000, "max_iter must lie in [0, 100000]");
    FT_ARG_CHECK(cfg->refine_steps == 0, "batches solve in binary64 (refine_steps must be 0)");
    if (!batch_has_sources(b)) {
        set_error("this batch has no built-in sources: run it with ft_batch_consume_run");
        return FT_E_ORDER;
    }
    const ft_status st = batch_run(b, cfg, x, bvec, reports, status, stream);
    if (st == FT_OK || st == FT_E_NOCONV || st == FT_E_NONFINITE) batch_mark_consumed(b);
    return st;
    FT_GUARD_END
}

ft_status ft_batch_consume_run(ft_batch* b, const ft_solve_cfg* cfg, const void* const* values, double* const* x,
                               double* const* bvec, ft_report* reports, int32_t* status, hipStream_t stream) {
    FT_GUARD_BEGIN
    clear_error();
    FT_ARG_CHECK(b && cfg && values && x && reports, "null argument");
    FT_ARG_CHECK(cfg->rtol >= 0.0 && std::isfinite(cfg->rtol), "rtol must be finite and >= 0");
    FT_ARG_CHECK(cfg->max_iter >= 0 && cfg->max_iter <= 100000, "max_iter must lie in [0, 100000]");
    FT_ARG_CHECK(cfg->refine_steps == 0, "batches solve in binary64 (refine_steps must be 0)");
    for (int k = 0; k < batch_count(b); ++k) {
        auto* T = static_cast<ft_target_ext*>(batch_target(b, k));
        const ft_sample_cfg* c = batch_cfg(b, k);
        FT_ARG_CHECK(values[k], "values[%d] is null", k);
        if (!T->sampled || !same_samples(T->sampled_cfg, *c)) {
            set_error("transfer %d: its target needs a prior ft_sample_points with the transfer's samples_per_elem, "
                      "seed, stream_id and point precision", k);
            return FT_E_ORDER;
        }
        if (c->alpha_mode != FT_ALPHA_FIXED) {
            set_error("transfer %d: batches use one fixed alpha per transfer", k);
            return FT_E_UNSUPPORTED;
        }
        FT_TRY(ensure_field_buffers(T, c->n_fields, stream));
    }
    const ft_status st = batch_run_values(b, cfg, values, x, bvec, reports, status, stream);
    if (st == FT_OK || st == FT_E_NOCONV || st == FT_E_NONFINITE) batch_mark_consumed(b);
    return st;
    FT_GUARD_END
}

ft_status ft_batch_autotune(ft_batch* b, const char* cache_path, int32_t* n_tuned, hipStream_t stream) {
    FT_GUARD_BEGIN
    clear_error();
    FT_ARG_CHECK(b, "batch is null");
    if (!batch_has_sources(b)) {
        set_error("the batch autotuner times the built-in route: this batch has no sources");
        return FT_E_ORDER;
    }
    return batch_autotune(b, cache_path, n_tuned, stream);
    FT_GUARD_END
}

ft_status ft_batch_variant(const ft_batch* b, int32_t k, int32_t* lanes_per_elem, int32_t* samples_per_lane) {
    clear_error();
    FT_ARG_CHECK(b && lanes_per_elem && samples_per_lane, "null argument");
    FT_ARG_CHECK(k >= 0 && k < batch_count(b), "transfer index %d out of range", k);
    batch_variant(b, k, lanes_per_elem, samples_per_lane);
    return FT_OK;
}

ft_status ft_batch_destroy(ft_batch* b) {
    if (!b) return FT_OK;
    batch_release(b);
    batch_delete(b);
    return FT_OK;
}

ft_status ft_source_create_p1(int32_t dim, int64_t n_nodes, const double* coords, int64_t n_elems,
                              const int32_t* conn, int32_t n_fields, const double* nodal_values, const int32_t* bins,
                              hipStream_t stream, ft_source** out) {
    FT_GUARD_BEGIN
    clear_error();
    FT_ARG_CHECK(out, "out is null");
    *out = nullptr;
    FT_ARG_CHECK(dim == 2 || dim == 3, "dim must be 2 or 3 (got %d)", dim);
    FT_ARG_CHECK(coords && conn && nodal_values, "coords, conn and nodal_values must be device pointers");
    FT_ARG_CHECK(n_nodes >= dim + 1 && n_nodes < INT32_MAX, "n_nodes out of range (%lld)", (long long)n_nodes);
    FT_ARG_CHECK(n_elems >= 1 && n_elems < INT32_MAX, "n_elems out of range (%lld)", (long long)n_elems);
    FT_ARG_CHECK(n_fields >= 1, "n_fields must be >= 1");
    if (bins)
        for (int c = 0; c < dim; ++c) FT_ARG_CHECK(bins[c] >= 0, "bins must be >= 0 (0 = default)");
    auto* S = new ft_source();
    S->dim = dim;
    S->n = n_nodes;
    S->E = n_elems;
    S->F = n_fields;
    const ft_status st = source_setup(S, coords, conn, nodal_values, bins, stream);
    if (st != FT_OK) {
        (void)hipStreamSynchronize(stream);
        source_release(S);
        delete S;
        return st;
    }
    *out = S;
    return FT_OK;
    FT_GUARD_END
}

ft_status ft_source_eval(ft_source* s, int64_t n_points, const void* points, int64_t ld, int32_t precision,
                         void* values, int64_t ld_out, int32_t* elem_ids, hipStream_t stream) {
    FT_GUARD_BEGIN
    clear_error();
    FT_ARG_CHECK(s, "source is null");
    FT_ARG_CHECK(n_points >= 0, "n_points must be >= 0");
    FT_ARG_CHECK(n_points == 0 || (points && values), "points and values must be device pointers");
    FT_ARG_CHECK(ld >= n_points && ld_out >= n_points, "leading dimensions must be >= n_points");
    FT_ARG_CHECK(precision == FT_F64 || precision == FT_F32, "precision must be FT_F64 or FT_F32");
    FT_ARG_CHECK(n_points < (int64_t(1) << 39), "n_points too large");
    return source_eval(s, 0, n_points, points, ld, precision, values, ld_out, elem_ids, stream, nullptr);
    FT_GUARD_END
}

ft_status ft_source_eval_queries(ft_source* s, int64_t n_nodes, int64_t n_points, const void* points, int64_t ld,
                                 int32_t precision, void* values, int64_t ld_out, int32_t* elem_ids,
                                 hipStream_t stream) {
    FT_GUARD_BEGIN
    clear_error();
    FT_ARG_CHECK(s, "source is null");
    FT_ARG_CHECK(n_points >= 0, "n_points must be >= 0");
    FT_ARG_CHECK(n_nodes >= 0 && n_nodes <= n_points, "n_nodes must lie in [0, n_points]");
    FT_ARG_CHECK(n_points == 0 || (points && values), "points and values must be device pointers");
    FT_ARG_CHECK(ld >= n_points && ld_out >= n_points, "leading dimensions must be >= n_points");
    FT_ARG_CHECK(precision == FT_F64 || precision == FT_F32, "precision must be FT_F64 or FT_F32");
    FT_ARG_CHECK(n_points < (int64_t(1) << 39), "n_points too large");
    return source_eval(s, n_nodes, n_points, points, ld, precision, values, ld_out, elem_ids, stream, nullptr);
    FT_GUARD_END
}

ft_status ft_source_eval_tiles(ft_source* s, int64_t n_nodes, int64_t n_elems, int32_t samples_per_elem,
                               const void* points, int64_t ld, int32_t precision, void* values, int32_t* elem_ids,
                               hipStream_t stream) {
    FT_GUARD_BEGIN
    clear_error();
    FT_ARG_CHECK(s, "source is null");
    FT_ARG_CHECK(n_nodes >= 0 && n_elems >= 0 && samples_per_elem >= 1, "sizes out of range");
    FT_ARG_CHECK(uint64_t(n_elems) * uint64_t(samples_per_elem) < (uint64_t(1) << 32),
                 "n_elems * samples_per_elem must stay below 2^32");
    const int64_t npts = n_nodes + n_elems * int64_t(samples_per_elem);
    FT_ARG_CHECK(npts == 0 || (points && values), "points and values must be device pointers");
    FT_ARG_CHECK(ld >= npts, "ld must be >= n_nodes + n_elems * samples_per_elem");
    FT_ARG_CHECK(precision == FT_F64 || precision == FT_F32, "precision must be FT_F64 or FT_F32");
    return source_eval_tiles(s, n_nodes, n_elems, samples_per_elem, points, ld, precision, values, elem_ids, stream);
    FT_GUARD_END
}

ft_status ft_source_autotune(ft_source* s, int64_t n_nodes, int64_t n_points, const void* points, int64_t ld,
                             int32_t precision, int32_t n_candidates, const int32_t* candidates, int32_t* bins_out,
                             hipStream_t stream) {
    FT_GUARD_BEGIN
    clear_error();
    FT_ARG_CHECK(s, "source is null");
    FT_ARG_CHECK(n_points >= 1 && points, "a sample of at least one point is needed");
    FT_ARG_CHECK(n_nodes >= 0 && n_nodes <= n_points, "n_nodes must lie in [0, n_points]");
    FT_ARG_CHECK(ld >= n_points, "ld must be >= n_points");
    FT_ARG_CHECK(precision == FT_F64 || precision == FT_F32, "precision must be FT_F64 or FT_F32");
    FT_ARG_CHECK(n_candidates >= 1 && n_candidates <= 64 && candidates, "1..64 candidates are needed");
    for (int c = 0; c < n_candidates; ++c)
        FT_ARG_CHECK(candidates[c] >= 1 && candidates[c] <= (1 << 20), "candidate %d out of range (%d)", c,
                     candidates[c]);
    FT_TRY(source_autotune(s, n_nodes, n_points, points, ld, precision, n_candidates, candidates, stream));
    if (bins_out)
        for (int c = 0; c < 3; ++c) bins_out[c] = s->nb[c];
    return FT_OK;
    FT_GUARD_END
}

ft_status ft_source_get_info(const ft_source* s, ft_source_info* info) {
    clear_error();
    FT_ARG_CHECK(s && info, "null argument");
    info->dim = s->dim;
    info->n_fields = s->F;
    info->n_nodes = s->n;
    info->n_elems = s->E;
    for (int c = 0; c < 3; ++c) info->bins[c] = s->nb[c];
    info->n_registrations = s->n_reg;
    return FT_OK;
}

ft_status ft_source_integral(ft_source* s, double* integrals, hipStream_t stream) {
    FT_GUARD_BEGIN
    clear_error();
    FT_ARG_CHECK(s && integrals, "null argument");
    return source_integral(s, integrals, stream);
    FT_GUARD_END
}

ft_status ft_source_stats(ft_source* s, int64_t* n_out_of_domain, hipStream_t stream) {
    FT_GUARD_BEGIN
    clear_error();
    FT_ARG_CHECK(s && n_out_of_domain, "null argument");
    FT_TRY_HIP(hipMemcpyAsync(s->h_counters, s->counters, sizeof(unsigned long long), hipMemcpyDeviceToHost, stream));
    FT_TRY_HIP(hipMemsetAsync(s->counters, 0, sizeof(unsigned long long), stream));
    FT_TRY_HIP(hipStreamSynchronize(stream));
    *n_out_of_domain = int64_t(s->h_counters[0]);
    return FT_OK;
    FT_GUARD_END
}

ft_status ft_source_destroy(ft_source* s) {
    if (!s) return FT_OK;
    source_release(s);
    delete s;
    return FT_OK;
}

int32_t ft_samples_for_tolerance(const ft_report* rep, int32_t samples_per_elem, double rel_tol) {
    if (!rep || samples_per_elem < 1 || !(rel_tol > 0.0) || std::isnan(rep->sum_b_stderr) || rep->sum_b_stderr < 0.0)
        return -1;
    const double target = rel_tol * std::fabs(rep->sum_b);
    if (rep->sum_b_stderr == 0.0 || !(target > 0.0)) return 1;
    const double r = rep->sum_b_stderr / target;
    const double n = std::ceil(double(samples_per_elem) * r * r);
    if (!(n < double(1 << 20))) return 1 << 20;
    return n < 1.0 ? 1 : int32_t(n);
}

int64_t ft_budget_for_tolerance(double weight_sum, double sum_b, double rel_tol) {
    if (!(rel_tol > 0.0) || !(weight_sum >= 0.0) || !std::isfinite(weight_sum) || !std::isfinite(sum_b)) return -1;
    const double target = rel_tol * std::fabs(sum_b);
    if (weight_sum == 0.0 || !(target > 0.0)) return 1;
    const double r = weight_sum / target;
    const double b = std::ceil(r * r);
    if (!(b < double(kMaxAllocTotal))) return kMaxAllocTotal;
    return b < 1.0 ? 1 : int64_t(b);
}

const char* ft_last_error(void) { return ft::last_error(); }

}  // extern "C"
