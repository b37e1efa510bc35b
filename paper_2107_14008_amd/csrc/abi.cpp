// C ABI of the short-range PM-FMM library: context, validation, planning,
// device upload, and the enqueueing of the forward and adjoint passes.
#include "pmfmm.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "device.h"
#include "plan.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                 \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(e_ == hipErrorOutOfMemory ? PMFMM_ENOMEM : PMFMM_EDEVICE,     \
                        std::string(#expr) + ": " + hipGetErrorString(e_));           \
    } while (0)

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t want) {
        if (want <= bytes && p != nullptr) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        if (want == 0) want = 16;
        hipError_t e = hipMalloc(&p, want);
        if (e == hipSuccess) bytes = want;
        return e;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <class T>
    T* as() const { return static_cast<T*>(p); }
};

bool valid_geometry(const pmfmm_params& p, std::string& why) {
    if (!(std::isfinite(p.box) && p.box > 0.0)) { why = "box must be finite and > 0"; return false; }
    if (!(std::isfinite(p.r_s) && p.r_s > 0.0)) { why = "r_s must be finite and > 0"; return false; }
    if (!(std::isfinite(p.r_cut) && p.r_cut > 0.0 && p.r_cut < 0.5 * p.box)) {
        why = "r_cut must satisfy 0 < r_cut < box / 2";
        return false;
    }
    if (!std::isfinite(p.G)) { why = "G must be finite"; return false; }
    if (!(std::isfinite(p.theta) && p.theta >= 0.0 && p.theta < 1.0)) {
        why = "theta must be in [0, 1)";
        return false;
    }
    if (p.max_leaf < 1 || p.max_leaf > 64) { why = "max_leaf must be in 1..64"; return false; }
    if (p.order > 6) { why = "order must be <= 6 (negative turns the far field off)"; return false; }
    return true;
}

bool valid_eval(const pmfmm_params& p, std::string& why) {
    if (p.precision != PMFMM_FP64 && p.precision != PMFMM_FP32) { why = "precision must be FP64 or FP32"; return false; }
    if (p.trunc != PMFMM_TRUNC_EXACT && p.trunc != PMFMM_TRUNC_TABLE) { why = "trunc must be EXACT or TABLE"; return false; }
    if (p.table_level < 0 || p.table_level > 4) { why = "table_level must be in 0..4"; return false; }
    if (p.table_round != PMFMM_ROUND_NEAREST && p.table_round != PMFMM_ROUND_FLOOR) { why = "table_round must be NEAREST or FLOOR"; return false; }
    const int max_tab = p.precision == PMFMM_FP64 ? 2048 : 4096;
    if (p.table_size < 16 || p.table_size > max_tab) {
        why = "table_size must be in 16.." + std::to_string(max_tab);
        return false;
    }
    if (p.chunk < 0) { why = "chunk must be >= 0"; return false; }
    if (p.wg_waves < 0 || p.wg_waves > 16) { why = "wg_waves must be in 0..16"; return false; }
    if (p.grid_wgs < 0) { why = "grid_wgs must be >= 0"; return false; }
    if (p.threads < 0) { why = "threads must be >= 0"; return false; }
    return true;
}

int mode_of(const pmfmm_params& p) {
    if (p.precision == PMFMM_FP64) return p.trunc == PMFMM_TRUNC_TABLE ? pmfmm::kFP64Table : pmfmm::kFP64Exact;
    return p.trunc == PMFMM_TRUNC_TABLE ? pmfmm::kFP32Table : pmfmm::kFP32Exact;
}

// Coefficients of Eq. (int) in table units e = (x - x_i) / h:
//   c_k = a_k(x_i) h^k with a_0 = T_i = erfc(x_i) - x_i E_i / 2,
//   a_1 = x_i^2 E_i, a_2 = -x_i (x_i^2 - 1) E_i,
//   a_3 = (2/3 x_i^4 - 5/3 x_i^2 + 1/3) E_i, a_4 = -x_i (x_i^4 / 3 - 3/2 x_i^2 + 1) E_i,
//   E_i = -4 exp(-x_i^2) / sqrt(pi), x_i = i h, h = 3 / n_tab.
std::vector<unsigned char> build_table(const pmfmm_params& p) {
    const int n = p.table_size;
    const double h = 3.0 / n;
    const double inv_sqrt_pi = 0.56418958354775628695;
    std::vector<double> c[5];
    for (auto& v : c) v.resize(n);
    for (int i = 0; i < n; ++i) {
        const double x = i * h, x2 = x * x;
        const double E = -4.0 * std::exp(-x2) * inv_sqrt_pi;
        const double a[5] = {std::erfc(x) - x * E / 2.0, x2 * E, -x * (x2 - 1.0) * E,
                             ((2.0 / 3.0) * x2 * x2 - (5.0 / 3.0) * x2 + 1.0 / 3.0) * E,
                             -x * ((1.0 / 3.0) * x2 * x2 - 1.5 * x2 + 1.0) * E};
        double hk = 1.0;
        for (int k = 0; k < 5; ++k) {
            c[k][i] = a[k] * hk;
            hk *= h;
        }
    }
    std::vector<unsigned char> out;
    if (p.precision == PMFMM_FP32) {
        out.resize((size_t)20 * n + 16);
        float* f4 = reinterpret_cast<float*>(out.data());
        float* f1 = reinterpret_cast<float*>(out.data() + 16 * (size_t)n);
        for (int i = 0; i < n; ++i) {
            for (int k = 0; k < 4; ++k) f4[4 * i + k] = (float)c[k][i];
            f1[i] = (float)c[4][i];
        }
    } else {
        out.resize((size_t)40 * n + 16);
        double* d01 = reinterpret_cast<double*>(out.data());
        double* d23 = reinterpret_cast<double*>(out.data() + 16 * (size_t)n);
        double* d4 = reinterpret_cast<double*>(out.data() + 32 * (size_t)n);
        for (int i = 0; i < n; ++i) {
            d01[2 * i] = c[0][i];
            d01[2 * i + 1] = c[1][i];
            d23[2 * i] = c[2][i];
            d23[2 * i + 1] = c[3][i];
            d4[i] = c[4][i];
        }
    }
    out.resize((out.size() + 15) / 16 * 16);
    return out;
}

}  // namespace

struct pmfmm_ctx {
    pmfmm_params p{};
    pmfmm::Plan plan;
    bool planned = false;
    bool built = false;
    int device = -1;
    int n_cu = 0;
    // device buffers
    DevBuf perm, leaf, leafc, js, items, queue, leaf_slot, partial, counter, boxes, table;
    DevBuf x64, x32, stage_pos, stage_mass, far;
    DevBuf cell, cell_aux, cellc, M, Lc, m2l_row, m2l_src, m2l_shift, level_cells;
    DevBuf w64, w32;
    std::vector<unsigned char> table_host;
    bool table_dirty = true;
    int last_mode = -1;
    size_t lds_bytes = 0;
    // timing
    hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    bool timed_fwd = false, timed_adj = false;

    ~pmfmm_ctx() {
        if (device >= 0) {
            (void)hipSetDevice(device);
            (void)hipDeviceSynchronize();
        }
        for (DevBuf* b : {&perm, &leaf, &leafc, &js, &items, &queue, &leaf_slot, &partial, &counter,
                          &boxes, &table, &x64, &x32, &stage_pos, &stage_mass, &far, &cell, &cell_aux,
                          &cellc, &M, &Lc, &m2l_row, &m2l_src, &m2l_shift, &level_cells, &w64, &w32})
            b->release();
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

namespace {

std::vector<pmfmm::BoxParams> one_box(const pmfmm_params& p) {
    return {pmfmm::BoxParams{p.box, p.r_s, p.r_cut, p.G, p.theta, p.max_leaf, p.order}};
}

int do_plan(pmfmm_ctx* ctx, const std::vector<pmfmm::BoxParams>& boxes,
            const std::vector<int64_t>& counts, const double* pos, const double* mass) {
    ctx->planned = false;
    ctx->built = false;
    std::string msg;
    try {
        msg = pmfmm::make_plan(ctx->plan, boxes, counts, pos, mass, ctx->p.threads);
        if (msg.empty()) pmfmm::make_items(ctx->plan, ctx->p.chunk);
    } catch (const std::bad_alloc&) {
        return fail(PMFMM_ENOMEM, "host allocation failed while planning");
    } catch (const std::exception& e) {
        return fail(PMFMM_EINVAL, e.what());
    }
    if (!msg.empty()) return fail(PMFMM_EINVAL, msg);
    ctx->planned = true;
    return PMFMM_OK;
}

int check_box_params(int32_t nbox, const pmfmm_params* per_box, const int64_t* counts,
                     const pmfmm_params& eval, std::vector<pmfmm::BoxParams>& boxes,
                     std::vector<int64_t>& cnt) {
    if (nbox < 1 || per_box == nullptr || counts == nullptr) return fail(PMFMM_EINVAL, "need at least one box");
    for (int b = 0; b < nbox; ++b) {
        std::string why;
        if (!valid_geometry(per_box[b], why)) return fail(PMFMM_EINVAL, "box " + std::to_string(b) + ": " + why);
        if (eval.trunc == PMFMM_TRUNC_TABLE && per_box[b].r_cut / (2.0 * per_box[b].r_s) > 3.0)
            return fail(PMFMM_EINVAL, "box " + std::to_string(b) + ": the table covers r <= 6 r_s only");
        if (counts[b] < 1) return fail(PMFMM_EINVAL, "box " + std::to_string(b) + ": needs at least one particle");
        const pmfmm_params& q = per_box[b];
        boxes.push_back(pmfmm::BoxParams{q.box, q.r_s, q.r_cut, q.G, q.theta, q.max_leaf, q.order});
        cnt.push_back(counts[b]);
    }
    return PMFMM_OK;
}

template <class T>
int upload(DevBuf& b, const std::vector<T>& v, hipStream_t s) {
    HIP_TRY(b.ensure(v.size() * sizeof(T)));
    if (!v.empty()) HIP_TRY(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return PMFMM_OK;
}

int upload_items(pmfmm_ctx* ctx, hipStream_t s) {
    const pmfmm::Plan& pl = ctx->plan;
    std::vector<int32_t> it(4 * pl.items.size());
    for (size_t k = 0; k < pl.items.size(); ++k) {
        it[4 * k] = pl.items[k].leaf;
        it[4 * k + 1] = pl.items[k].t0;
        it[4 * k + 2] = pl.items[k].t1;
        it[4 * k + 3] = pl.items[k].slot;
    }
    int rc;
    if ((rc = upload(ctx->items, it, s))) return rc;
    if ((rc = upload(ctx->queue, pl.queue, s))) return rc;
    if ((rc = upload(ctx->leaf_slot, pl.leaf_slot_begin, s))) return rc;
    HIP_TRY(ctx->partial.ensure(std::max<size_t>(1, pl.items.size()) * 4 * 64 * sizeof(double)));
    HIP_TRY(hipStreamSynchronize(s));
    return PMFMM_OK;
}

int upload_table(pmfmm_ctx* ctx, hipStream_t s) {
    if (!ctx->table_dirty) return PMFMM_OK;
    ctx->table_host = build_table(ctx->p);
    int rc = upload(ctx->table, ctx->table_host, s);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(s));
    ctx->table_dirty = false;
    return PMFMM_OK;
}

std::vector<pmfmm::BoxDev> box_table(const pmfmm_ctx* ctx) {
    std::vector<pmfmm::BoxDev> out;
    for (const auto& b : ctx->plan.boxes) {
        pmfmm::BoxDev d{};
        d.L = b.box;
        d.alpha = 1.0 / (2.0 * b.r_s);
        d.rc2 = b.r_cut * b.r_cut;
        d.G = b.G;
        d.alpha_f = (float)d.alpha;
        d.rc2_f = (float)d.rc2;
        d.tab_scale = d.alpha * (ctx->p.table_size / 3.0);
        d.tab_scale_f = (float)d.tab_scale;
        d.order = (b.order >= 0 && b.theta > 0.0) ? b.order : -1;
        out.push_back(d);
    }
    return out;
}

int do_upload(pmfmm_ctx* ctx, const double* pos, const double* mass, int32_t on_device, hipStream_t s) {
    const pmfmm::Plan& pl = ctx->plan;
    HIP_TRY(hipGetDevice(&ctx->device));
    HIP_TRY(hipDeviceGetAttribute(&ctx->n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device));
    const int64_t n = pl.n, nl = (int64_t)pl.leaf_count.size();
    std::vector<int32_t> leaf(4 * nl);
    std::vector<double> leafc(4 * nl);
    for (int64_t l = 0; l < nl; ++l) {
        const pmfmm::Cell& c = pl.cells[pl.leaf_cell[l]];
        leaf[4 * l] = c.first;
        leaf[4 * l + 1] = c.count;
        leaf[4 * l + 2] = c.box;
        leaf[4 * l + 3] = pl.leaf_cell[l];
        for (int a = 0; a < 3; ++a) leafc[4 * l + a] = 0.5 * (c.lo[a] + c.hi[a]);
        leafc[4 * l + 3] = 0.0;
    }
    std::vector<int32_t> js(pl.p2p_j.size());
    for (size_t t = 0; t < js.size(); ++t) js[t] = (pl.p2p_j[t] << 5) | pl.p2p_shift[t];
    int rc;
    if ((rc = upload(ctx->perm, pl.perm, s))) return rc;
    if ((rc = upload(ctx->leaf, leaf, s))) return rc;
    if ((rc = upload(ctx->leafc, leafc, s))) return rc;
    if ((rc = upload(ctx->js, js, s))) return rc;
    if ((rc = upload(ctx->boxes, box_table(ctx), s))) return rc;
    HIP_TRY(ctx->counter.ensure(64));
    HIP_TRY(ctx->x64.ensure((size_t)n * 32));
    HIP_TRY(ctx->x32.ensure((size_t)n * 16));
    const double* src_pos = pos;
    const double* src_mass = mass;
    if (!on_device) {
        if ((rc = upload(ctx->stage_pos, pl.pos, s))) return rc;
        if ((rc = upload(ctx->stage_mass, pl.mass, s))) return rc;
        src_pos = ctx->stage_pos.as<double>();
        src_mass = ctx->stage_mass.as<double>();
    }
    pmfmm::GatherArgs g{src_pos, src_mass, ctx->perm.as<int32_t>(), ctx->leaf.as<int4>(),
                        ctx->leafc.as<double4>(), ctx->boxes.as<pmfmm::BoxDev>(), ctx->x64.as<double4>(),
                        ctx->x32.as<float4>(), (int32_t)nl};
    HIP_TRY(pmfmm::launch_gather(g, nullptr, s));
    if ((rc = upload_items(ctx, s))) return rc;
    ctx->table_dirty = true;
    if ((rc = upload_table(ctx, s))) return rc;
    if (pl.far_field) {
        // far-field arrays
        const int64_t nc = (int64_t)pl.cells.size();
        std::vector<int32_t> cell(4 * nc), aux(4 * nc);
        std::vector<double> cc(4 * nc);
        for (int64_t k = 0; k < nc; ++k) {
            const pmfmm::Cell& c = pl.cells[k];
            cell[4 * k] = c.first;
            cell[4 * k + 1] = c.count;
            cell[4 * k + 2] = c.parent;
            cell[4 * k + 3] = c.leaf;
            aux[4 * k] = c.child[0];
            aux[4 * k + 1] = c.child[1];
            aux[4 * k + 2] = c.box;
            aux[4 * k + 3] = c.depth;
            for (int a = 0; a < 3; ++a) cc[4 * k + a] = 0.5 * (c.lo[a] + c.hi[a]);
            cc[4 * k + 3] = 0.0;
        }
        if ((rc = upload(ctx->cell, cell, s))) return rc;
        if ((rc = upload(ctx->cell_aux, aux, s))) return rc;
        if ((rc = upload(ctx->cellc, cc, s))) return rc;
        if ((rc = upload(ctx->m2l_row, pl.m2l_row, s))) return rc;
        if ((rc = upload(ctx->m2l_src, pl.m2l_src, s))) return rc;
        if ((rc = upload(ctx->m2l_shift, pl.m2l_shift, s))) return rc;
        if ((rc = upload(ctx->level_cells, pl.cells_by_depth, s))) return rc;
        const int nco = pmfmm::n_coef(pl.max_order);
        HIP_TRY(ctx->M.ensure((size_t)nc * nco * sizeof(double)));
        HIP_TRY(ctx->Lc.ensure((size_t)nc * nco * sizeof(double)));
        HIP_TRY(ctx->far.ensure((size_t)n * 3 * sizeof(double)));
    }
    HIP_TRY(hipStreamSynchronize(s));
    ctx->built = true;
    return PMFMM_OK;
}

int default_wg_waves(int mode) {
    return mode == pmfmm::kFP64Table ? 16 : 4;
}

int run_far(pmfmm_ctx* ctx, hipStream_t s) {
    const pmfmm::Plan& pl = ctx->plan;
    const int64_t nc = (int64_t)pl.cells.size();
    pmfmm::FarArgs f{};
    f.x64 = ctx->x64.as<double4>();
    f.leaf = ctx->leaf.as<int4>();
    f.leafc = ctx->leafc.as<double4>();
    f.cell = ctx->cell.as<int4>();
    f.cell_aux = ctx->cell_aux.as<int4>();
    f.cellc = ctx->cellc.as<double4>();
    f.m2l_row = ctx->m2l_row.as<int32_t>();
    f.m2l_src = ctx->m2l_src.as<int32_t>();
    f.m2l_shift = ctx->m2l_shift.as<int32_t>();
    f.boxes = ctx->boxes.as<pmfmm::BoxDev>();
    f.M = ctx->M.as<double>();
    f.Lc = ctx->Lc.as<double>();
    f.far = ctx->far.as<double>();
    f.n_cells = (int32_t)nc;
    f.n_leaves = (int32_t)pl.leaf_count.size();
    f.order = pl.max_order;
    f.ncoef = pmfmm::n_coef(pl.max_order);
    HIP_TRY(pmfmm::launch_zero_f64(f.M, nc * f.ncoef, s));
    HIP_TRY(pmfmm::launch_p2m(f, s));
    const int nd = (int)pl.depth_begin.size() - 1;
    for (int d = nd - 2; d >= 0; --d) {   // parents of the deepest level first
        f.level_cells = ctx->level_cells.as<int32_t>() + pl.depth_begin[d];
        f.n_level = pl.depth_begin[d + 1] - pl.depth_begin[d];
        HIP_TRY(pmfmm::launch_m2m_level(f, s));
    }
    HIP_TRY(pmfmm::launch_m2l(f, s));
    for (int d = 1; d < nd; ++d) {
        f.level_cells = ctx->level_cells.as<int32_t>() + pl.depth_begin[d];
        f.n_level = pl.depth_begin[d + 1] - pl.depth_begin[d];
        HIP_TRY(pmfmm::launch_l2l_level(f, s));
    }
    HIP_TRY(pmfmm::launch_l2p(f, s));
    return PMFMM_OK;
}

int ensure_events(pmfmm_ctx* ctx) {
    for (auto& e : ctx->ev)
        if (!e) HIP_TRY(hipEventCreate(&e));
    return PMFMM_OK;
}

}  // namespace

extern "C" {

void pmfmm_params_init(pmfmm_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->box = 100.0;
    p->r_s = 3.75;
    p->r_cut = 4.5 * 3.75;
    p->G = 1.0;
    p->theta = 0.0;
    p->max_leaf = 64;
    p->order = 4;
    p->precision = PMFMM_FP64;
    p->trunc = PMFMM_TRUNC_EXACT;
    p->table_size = 2048;
    p->table_level = 4;
    p->table_round = PMFMM_ROUND_NEAREST;
}

const char* pmfmm_version(void) { return "pmfmm-mi355x 0.1"; }

const char* pmfmm_last_error(void) { return g_err.c_str(); }

int pmfmm_create(const pmfmm_params* p, pmfmm_ctx** out) {
    if (!p || !out) return fail(PMFMM_EINVAL, "null argument");
    std::string why;
    if (!valid_geometry(*p, why) || !valid_eval(*p, why)) return fail(PMFMM_EINVAL, why);
    if (p->trunc == PMFMM_TRUNC_TABLE && p->r_cut / (2.0 * p->r_s) > 3.0)
        return fail(PMFMM_EINVAL, "the table covers r <= 6 r_s only");
    pmfmm_ctx* c = new (std::nothrow) pmfmm_ctx();
    if (!c) return fail(PMFMM_ENOMEM, "context allocation failed");
    c->p = *p;
    *out = c;
    return PMFMM_OK;
}

void pmfmm_destroy(pmfmm_ctx* ctx) { delete ctx; }

int pmfmm_plan(pmfmm_ctx* ctx, int64_t n, const double* pos, const double* mass) {
    if (!ctx || !pos || !mass) return fail(PMFMM_EINVAL, "null argument");
    if (n < 1) return fail(PMFMM_EINVAL, "n must be >= 1");
    return do_plan(ctx, one_box(ctx->p), {n}, pos, mass);
}

int pmfmm_plan_batch(pmfmm_ctx* ctx, int32_t nbox, const pmfmm_params* per_box,
                     const int64_t* counts, const double* pos, const double* mass) {
    if (!ctx || !pos || !mass) return fail(PMFMM_EINVAL, "null argument");
    std::vector<pmfmm::BoxParams> boxes;
    std::vector<int64_t> cnt;
    int rc = check_box_params(nbox, per_box, counts, ctx->p, boxes, cnt);
    if (rc) return rc;
    return do_plan(ctx, boxes, cnt, pos, mass);
}

static int build_common(pmfmm_ctx* ctx, const std::vector<pmfmm::BoxParams>& boxes,
                        const std::vector<int64_t>& cnt, const double* pos, const double* mass,
                        int32_t on_device, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    int64_t n = 0;
    for (int64_t c : cnt) n += c;
    const double* hp = pos;
    const double* hm = mass;
    std::vector<double> tmp_pos, tmp_mass;
    if (on_device) {
        tmp_pos.resize(3 * (size_t)n);
        tmp_mass.resize((size_t)n);
        HIP_TRY(hipMemcpyAsync(tmp_pos.data(), pos, tmp_pos.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(tmp_mass.data(), mass, tmp_mass.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        hp = tmp_pos.data();
        hm = tmp_mass.data();
    }
    int rc = do_plan(ctx, boxes, cnt, hp, hm);
    if (rc) return rc;
    return do_upload(ctx, pos, mass, on_device, s);
}

int pmfmm_build(pmfmm_ctx* ctx, int64_t n, const double* pos, const double* mass, int32_t on_device,
                void* stream) {
    if (!ctx || !pos || !mass) return fail(PMFMM_EINVAL, "null argument");
    if (n < 1) return fail(PMFMM_EINVAL, "n must be >= 1");
    return build_common(ctx, one_box(ctx->p), {n}, pos, mass, on_device, stream);
}

int pmfmm_build_batch(pmfmm_ctx* ctx, int32_t nbox, const pmfmm_params* per_box, const int64_t* counts,
                      const double* pos, const double* mass, int32_t on_device, void* stream) {
    if (!ctx || !pos || !mass) return fail(PMFMM_EINVAL, "null argument");
    std::vector<pmfmm::BoxParams> boxes;
    std::vector<int64_t> cnt;
    int rc = check_box_params(nbox, per_box, counts, ctx->p, boxes, cnt);
    if (rc) return rc;
    return build_common(ctx, boxes, cnt, pos, mass, on_device, stream);
}

int pmfmm_set_eval(pmfmm_ctx* ctx, const pmfmm_params* p) {
    if (!ctx || !p) return fail(PMFMM_EINVAL, "null argument");
    std::string why;
    if (!valid_eval(*p, why)) return fail(PMFMM_EINVAL, why);
    if (p->trunc == PMFMM_TRUNC_TABLE && ctx->planned)
        for (const auto& b : ctx->plan.boxes)
            if (b.r_cut / (2.0 * b.r_s) > 3.0) return fail(PMFMM_EINVAL, "the table covers r <= 6 r_s only");
    const bool table_change = p->precision != ctx->p.precision || p->table_size != ctx->p.table_size;
    const bool chunk_change = p->chunk != ctx->p.chunk;
    ctx->p.precision = p->precision;
    ctx->p.trunc = p->trunc;
    ctx->p.table_size = p->table_size;
    ctx->p.table_level = p->table_level;
    ctx->p.table_round = p->table_round;
    ctx->p.chunk = p->chunk;
    ctx->p.wg_waves = p->wg_waves;
    ctx->p.grid_wgs = p->grid_wgs;
    ctx->p.timing = p->timing;
    if (table_change) ctx->table_dirty = true;
    if (ctx->planned && chunk_change) {
        pmfmm::make_items(ctx->plan, ctx->p.chunk);
        if (ctx->built) {
            int rc = upload_items(ctx, nullptr);
            if (rc) return rc;
        }
    }
    if (ctx->built) {
        // per-box constants depend on table_size
        int rc = upload(ctx->boxes, box_table(ctx), nullptr);
        if (rc) return rc;
        HIP_TRY(hipStreamSynchronize(nullptr));
    }
    return PMFMM_OK;
}

int pmfmm_forward(pmfmm_ctx* ctx, double* acc, void* stream) {
    if (!ctx || !acc) return fail(PMFMM_EINVAL, "null argument");
    if (!ctx->built) return fail(PMFMM_ESTATE, "forward before build");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = upload_table(ctx, s);
    if (rc) return rc;
    const pmfmm::Plan& pl = ctx->plan;
    const int mode = mode_of(ctx->p);
    const bool timing = ctx->p.timing != 0;
    if (timing) {
        if ((rc = ensure_events(ctx))) return rc;
        HIP_TRY(hipEventRecord(ctx->ev[0], s));
    }
    if (pl.far_field) {
        if ((rc = run_far(ctx, s))) return rc;
    }
    HIP_TRY(pmfmm::launch_zero_i32(ctx->counter.as<int32_t>(), 1, s));
    if (timing) HIP_TRY(hipEventRecord(ctx->ev[1], s));
    pmfmm::P2PArgs a{};
    a.x64 = ctx->x64.as<double4>();
    a.x32 = ctx->x32.as<float4>();
    a.leaf = ctx->leaf.as<int4>();
    a.leafc = ctx->leafc.as<double4>();
    a.p2p_js = ctx->js.as<int32_t>();
    a.items = ctx->items.as<int4>();
    a.queue = ctx->queue.as<int32_t>();
    a.n_items = (int32_t)pl.items.size();
    a.counter = ctx->counter.as<int32_t>();
    a.partial = ctx->partial.as<double>();
    a.boxes = ctx->boxes.as<pmfmm::BoxDev>();
    a.table = ctx->table.p;
    a.n_tab = ctx->p.table_size;
    a.level = ctx->p.table_level;
    a.round_floor = ctx->p.table_round == PMFMM_ROUND_FLOOR;
    const bool tab = mode == pmfmm::kFP32Table || mode == pmfmm::kFP64Table;
    const size_t lds = tab ? ctx->table_host.size() : 0;
    const int wg = ctx->p.wg_waves > 0 ? ctx->p.wg_waves : default_wg_waves(mode);
    int grid = ctx->p.grid_wgs;
    if (grid <= 0) grid = ctx->n_cu * pmfmm::p2p_blocks_per_cu(mode, wg, lds);
    HIP_TRY(pmfmm::launch_p2p(mode, a, wg, grid, lds, s));
    if (timing) HIP_TRY(hipEventRecord(ctx->ev[2], s));
    pmfmm::ReduceArgs r{ctx->leaf.as<int4>(), ctx->leaf_slot.as<int32_t>(), ctx->partial.as<double>(),
                        pl.far_field ? ctx->far.as<double>() : nullptr, ctx->perm.as<int32_t>(),
                        ctx->boxes.as<pmfmm::BoxDev>(), acc, (int32_t)pl.leaf_count.size()};
    HIP_TRY(pmfmm::launch_reduce(r, s));
    if (timing) {
        HIP_TRY(hipEventRecord(ctx->ev[3], s));
        ctx->timed_fwd = true;
    }
    return PMFMM_OK;
}

int pmfmm_get_lists(const pmfmm_ctx* ctx, pmfmm_lists* out) {
    if (!ctx || !out) return fail(PMFMM_EINVAL, "null argument");
    if (!ctx->planned) return fail(PMFMM_ESTATE, "no plan");
    const pmfmm::Plan& pl = ctx->plan;
    out->n = pl.n;
    out->n_boxes = (int64_t)pl.boxes.size();
    out->n_leaves = (int64_t)pl.leaf_count.size();
    out->n_cells = (int64_t)pl.cells.size();
    out->n_p2p = (int64_t)pl.p2p_j.size();
    out->n_m2l = (int64_t)pl.m2l_src.size();
    out->n_items = (int64_t)pl.items.size();
    out->candidate_pairs = pl.candidate_pairs;
    out->perm = pl.perm.data();
    out->box_first_leaf = pl.box_first_leaf.data();
    out->box_first_cell = pl.box_first_cell.data();
    out->leaf_first = pl.leaf_first.data();
    out->leaf_count = pl.leaf_count.data();
    out->leaf_cell = pl.leaf_cell.data();
    out->cell_first = pl.cell_first.data();
    out->cell_count = pl.cell_count.data();
    out->cell_child = pl.cell_child.data();
    out->cell_lo = pl.cell_lo.data();
    out->cell_hi = pl.cell_hi.data();
    out->p2p_row = pl.p2p_row.data();
    out->p2p_j = pl.p2p_j.data();
    out->p2p_shift = pl.p2p_shift.data();
    out->m2l_row = pl.m2l_row.data();
    out->m2l_src = pl.m2l_src.data();
    out->m2l_shift = pl.m2l_shift.data();
    return PMFMM_OK;
}

int pmfmm_get_timings(const pmfmm_ctx* ctx, pmfmm_timings* out) {
    if (!ctx || !out) return fail(PMFMM_EINVAL, "null argument");
    if (!ctx->timed_fwd && !ctx->timed_adj) return fail(PMFMM_ESTATE, "nothing timed (params.timing = 0?)");
    std::memset(out, 0, sizeof(*out));
    float ms = 0.f;
    if (ctx->timed_fwd) {
        HIP_TRY(hipEventSynchronize(ctx->ev[3]));
        HIP_TRY(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]));
        out->far_ms = ms;
        HIP_TRY(hipEventElapsedTime(&ms, ctx->ev[1], ctx->ev[2]));
        out->p2p_ms = ms;
        HIP_TRY(hipEventElapsedTime(&ms, ctx->ev[2], ctx->ev[3]));
        out->reduce_ms = ms;
        HIP_TRY(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[3]));
        out->total_ms = ms;
    }
    if (ctx->timed_adj) {
        HIP_TRY(hipEventSynchronize(ctx->ev[5]));
        HIP_TRY(hipEventElapsedTime(&ms, ctx->ev[4], ctx->ev[5]));
        out->adjoint_ms = ms;
    }
    return PMFMM_OK;
}

int pmfmm_adjoint(pmfmm_ctx* ctx, const double* w, double* grad_pos, double* grad_mass, void* stream) {
    if (!ctx || !w || !grad_pos || !grad_mass) return fail(PMFMM_EINVAL, "null argument");
    if (!ctx->built) return fail(PMFMM_ESTATE, "adjoint before build");
    if (ctx->plan.far_field) return fail(PMFMM_EUNSUPPORTED, "adjoint covers the P2P-only force (far field off)");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const pmfmm::Plan& pl = ctx->plan;
    const int64_t n = pl.n;
    HIP_TRY(ctx->w64.ensure((size_t)n * 32));
    HIP_TRY(ctx->w32.ensure((size_t)n * 16));
    HIP_TRY(pmfmm::launch_gather_w(w, ctx->perm.as<int32_t>(), ctx->w64.as<double4>(), ctx->w32.as<float4>(),
                                   (int32_t)n, s));
    HIP_TRY(pmfmm::launch_zero_i32(ctx->counter.as<int32_t>(), 1, s));
    const bool timing = ctx->p.timing != 0;
    if (timing) {
        int rc = ensure_events(ctx);
        if (rc) return rc;
        HIP_TRY(hipEventRecord(ctx->ev[4], s));
    }
    pmfmm::AdjArgs a{};
    a.x64 = ctx->x64.as<double4>();
    a.x32 = ctx->x32.as<float4>();
    a.w64 = ctx->w64.as<double4>();
    a.w32 = ctx->w32.as<float4>();
    a.leaf = ctx->leaf.as<int4>();
    a.leafc = ctx->leafc.as<double4>();
    a.p2p_js = ctx->js.as<int32_t>();
    a.items = ctx->items.as<int4>();
    a.queue = ctx->queue.as<int32_t>();
    a.n_items = (int32_t)pl.items.size();
    a.counter = ctx->counter.as<int32_t>();
    a.partial = ctx->partial.as<double>();
    a.boxes = ctx->boxes.as<pmfmm::BoxDev>();
    const int mode = mode_of(ctx->p);
    const int wg = ctx->p.wg_waves > 0 ? ctx->p.wg_waves : 4;
    int grid = ctx->p.grid_wgs;
    if (grid <= 0) grid = ctx->n_cu * pmfmm::adjoint_blocks_per_cu(mode, wg, 0);
    HIP_TRY(pmfmm::launch_adjoint(mode, a, wg, grid, 0, s));
    if (timing) {
        HIP_TRY(hipEventRecord(ctx->ev[5], s));
        ctx->timed_adj = true;
    }
    pmfmm::AdjReduceArgs r{ctx->leaf.as<int4>(), ctx->leaf_slot.as<int32_t>(), ctx->partial.as<double>(),
                           ctx->perm.as<int32_t>(), ctx->boxes.as<pmfmm::BoxDev>(), grad_pos, grad_mass,
                           (int32_t)pl.leaf_count.size()};
    HIP_TRY(pmfmm::launch_adj_reduce(r, s));
    return PMFMM_OK;
}

}  // extern "C"
