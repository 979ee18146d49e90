// C ABI of libsmm: contexts, problems, device tables and the SMM outer loop.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/smm_cnn.h"
#include "api_internal.hpp"
#include "cg_smm.hpp"
#include "mg_internal.hpp"

using namespace smm;

int smm::fail(smm_ctx* c, int code, const std::string& msg) {
    if (c) c->last_error = msg;
    return code;
}

// ---------------------------------------------------------------------------
// Work memory of smm_apply_G_noalloc: one fixed array per device, for callers
// that cannot allocate.  In host code `scratch` only names the symbol; its
// device address is looked up once per device (with that device current)
// when a context is created there, and only that address is ever passed to
// kernels and copies.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kScratchBytes = size_t(32) << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// the calling thread's current device must be `device`
int scratch_lookup(int device) {
    if (device < 0 || device >= kMaxDevices) return SMM_OK;  // the no-allocation entry point refuses it
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return SMM_OK;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return SMM_EHIP;
    g_scratch_ptr[device] = ptr;
    return SMM_OK;
}
}  // namespace

extern "C" {

const char* smm_strerror(int code) {
    switch (code) {
        case SMM_OK: return "ok";
        case SMM_EINVAL: return "invalid argument";
        case SMM_ENOMEM: return "out of memory";
        case SMM_EHIP: return "HIP runtime error";
        case SMM_ENOCONV: return "outer iteration did not converge";
        case SMM_ENAN: return "NaN or Inf in the outer residual";
        case SMM_EBREAKDOWN: return "CG breakdown (operator not positive definite)";
        case SMM_EUNSUPPORTED: return "unsupported input";
        case SMM_ESTATE: return "call order violated";
        default: return "unknown status";
    }
}

int smm_ctx_create(int device, void* hip_stream, smm_ctx** out) {
    if (!out) return SMM_EINVAL;
    smm_ctx* c = new (std::nothrow) smm_ctx();
    if (!c) return SMM_ENOMEM;
    c->device = device;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    if (device >= 0) {
        int cnt = 0;
        if (hipGetDeviceCount(&cnt) != hipSuccess || device >= cnt) {
            delete c;
            return SMM_EHIP;
        }
        if (hipSetDevice(device) != hipSuccess || scratch_lookup(device) != SMM_OK) {
            delete c;
            return SMM_EHIP;
        }
    }
    *out = c;
    return SMM_OK;
}

int smm_ctx_destroy(smm_ctx* ctx) {
    delete ctx;
    return SMM_OK;
}

const char* smm_last_error(smm_ctx* ctx) { return ctx ? ctx->last_error.c_str() : ""; }

}  // extern "C"

// Directions and weights of a quadrature descriptor (Sec. 4).
static int quad_from_desc(smm_ctx* ctx, const smm_quad_desc* q, Problem& P) {
    if (!q) return fail(ctx, SMM_EINVAL, "null quadrature descriptor");
    if (q->kind == SMM_QUAD_LEVEL_SYMMETRIC) {
        P.sn = q->sn_order;
        if (level_symmetric(q->sn_order, P.omega, P.w) != 0)
            return fail(ctx, SMM_EINVAL, "S_N order must be 4, 6, 8, 10 or 12");
        P.nd = (int)P.w.size();
        return SMM_OK;
    }
    if (q->kind != SMM_QUAD_EXPLICIT) return fail(ctx, SMM_EINVAL, "unknown quadrature kind");
    if (q->n_dir < 1 || q->n_dir > 4096 || !q->omega || !q->w)
        return fail(ctx, SMM_EINVAL, "explicit quadrature: n_dir in 1..4096 and both arrays required");
    double sw = 0;
    for (int d = 0; d < q->n_dir; ++d) {
        const double* o = &q->omega[d * 3];
        const double nrm = std::sqrt(o[0] * o[0] + o[1] * o[1] + o[2] * o[2]);
        if (!(std::fabs(nrm - 1.0) <= 1e-12) || !(o[2] >= 0.0) || !(q->w[d] > 0.0) || !std::isfinite(q->w[d]))
            return fail(ctx, SMM_EINVAL, "explicit quadrature: direction " + std::to_string(d) +
                                             " is not a unit vector with Omega_z >= 0 and a positive weight");
        if (o[0] == 0.0 || o[1] == 0.0)
            return fail(ctx, SMM_EUNSUPPORTED, "explicit quadrature: direction " + std::to_string(d) +
                                                   " has a zero in-plane component");
        sw += q->w[d];
    }
    const double fourpi = 16.0 * std::atan(1.0);
    if (!(std::fabs(sw - fourpi) <= 1e-12 * fourpi))
        return fail(ctx, SMM_EINVAL, "explicit quadrature: weights must sum to 4 pi");
    P.sn = 0;
    P.nd = q->n_dir;
    P.omega.assign(q->omega, q->omega + 3 * (size_t)q->n_dir);
    P.w.assign(q->w, q->w + q->n_dir);
    P.quad_explicit = true;
    return SMM_OK;
}

// Geometry set-up shared by the creation calls (P's sizes, mesh data and
// quadrature filled in).
static int create_common(smm_ctx* ctx, smm_problem* pr, smm_problem** out) {
    Problem& P = pr->P;
    std::string err;
    int rc = setup_geometry(P, err, false);
    if (rc != SMM_OK) {
        delete pr;
        return fail(ctx, rc, err);
    }
    // curved or irregular meshes need the per-element quadrature data and the
    // sweep graph at once; uniform Cartesian meshes build them only on demand
    if (!P.cartesian && (rc = ensure_heavy(P, &err)) != SMM_OK) {
        delete pr;
        return fail(ctx, rc, err.empty() ? std::string("geometry setup failed") : err);
    }
    P.q.assign((size_t)P.ne * P.n, 0.0);
    *out = pr;
    return SMM_OK;
}

static int create_structured(smm_ctx* ctx, const smm_mesh_desc* mesh, int p, const smm_quad_desc* quad,
                             smm_problem** out) {
    if (!ctx || !mesh || !out || !mesh->ctrl) return fail(ctx, SMM_EINVAL, "null argument");
    if (p < 1 || p > 4) return fail(ctx, SMM_EINVAL, "p must be in 1..4");
    if (mesh->nx < 1 || mesh->ny < 1 || mesh->m < 1 || mesh->m > 6)
        return fail(ctx, SMM_EINVAL, "bad mesh sizes");
    smm_problem* pr = new (std::nothrow) smm_problem();
    if (!pr) return SMM_ENOMEM;
    Problem& P = pr->P;
    P.ctx = ctx;
    P.nx = mesh->nx;
    P.ny = mesh->ny;
    P.m = mesh->m;
    P.p = p;
    P.nb = p + 1;
    P.n = P.nb * P.nb;
    P.nq = p + mesh->m + 1;
    P.ne = P.nx * P.ny;
    int rc = quad_from_desc(ctx, quad, P);
    if (rc) {
        delete pr;
        return rc;
    }
    const size_t nctrl = (size_t)(P.ny * P.m + 1) * (P.nx * P.m + 1) * 2;
    P.ctrl.assign(mesh->ctrl, mesh->ctrl + nctrl);
    return create_common(ctx, pr, out);
}

extern "C" {

int smm_problem_create(smm_ctx* ctx, const smm_mesh_desc* mesh, int p, int sn_order, smm_problem** out) {
    smm_quad_desc q{SMM_QUAD_LEVEL_SYMMETRIC, sn_order, 0, nullptr, nullptr};
    return create_structured(ctx, mesh, p, &q, out);
}

int smm_problem_create_q(smm_ctx* ctx, const smm_mesh_desc* mesh, int p, const smm_quad_desc* quad,
                         smm_problem** out) {
    return create_structured(ctx, mesh, p, quad, out);
}

int smm_problem_create_general(smm_ctx* ctx, const smm_mesh_general_desc* mesh, int p, const smm_quad_desc* quad,
                               smm_problem** out) {
    if (!ctx || !mesh || !out || !mesh->ctrl || !mesh->nbr) return fail(ctx, SMM_EINVAL, "null argument");
    if (p < 1 || p > 4) return fail(ctx, SMM_EINVAL, "p must be in 1..4");
    if (mesh->n_elem < 1 || mesh->m < 1 || mesh->m > 6) return fail(ctx, SMM_EINVAL, "bad mesh sizes");
    smm_problem* pr = new (std::nothrow) smm_problem();
    if (!pr) return SMM_ENOMEM;
    Problem& P = pr->P;
    P.ctx = ctx;
    P.general = true;
    P.ne = mesh->n_elem;
    P.nx = mesh->n_elem;
    P.ny = 1;
    P.m = mesh->m;
    P.p = p;
    P.nb = p + 1;
    P.n = P.nb * P.nb;
    P.nq = p + mesh->m + 1;
    int rc = quad_from_desc(ctx, quad, P);
    if (rc) {
        delete pr;
        return rc;
    }
    const size_t mm = (size_t)(P.m + 1) * (P.m + 1);
    P.ctrl_e.assign(mesh->ctrl, mesh->ctrl + (size_t)P.ne * mm * 2);
    P.nbr_in.assign(mesh->nbr, mesh->nbr + (size_t)P.ne * 4);
    for (int v : P.nbr_in)
        if (v < -1 || v >= P.ne) {
            delete pr;
            return fail(ctx, SMM_EINVAL, "neighbour index out of range");
        }
    if (mesh->bdr_attr) P.bdr_attr_in.assign(mesh->bdr_attr, mesh->bdr_attr + (size_t)P.ne * 4);
    return create_common(ctx, pr, out);
}

static void dev_free(Dev& D) {
    for (auto& e : D.ev)
        if (e) (void)hipEventDestroy(e);
    for (auto& g : D.cg_graphs) (void)hipGraphExecDestroy(g.second);
    if (D.cg_cap) (void)hipStreamDestroy(D.cg_cap);
    for (void* ptr : D.allocs) (void)hipFree(ptr);
    D.allocs.clear();
    D = Dev();
}

int smm_problem_destroy(smm_problem* prob) {
    if (!prob) return SMM_OK;
    batch_release_single(prob);
    dev_free(prob->D);
    delete prob;
    return SMM_OK;
}

int smm_get_dims(const smm_problem* prob, smm_problem_dims* out) {
    if (!prob || !out) return SMM_EINVAL;
    const Problem& P = prob->P;
    out->n_elem = P.ne;
    out->n_node = P.n;
    out->n_dir = P.nd;
    out->n_bface = P.nbf;
    out->nq = P.nq;
    out->cartesian = P.cartesian ? 1 : 0;
    out->n_material = P.nmat;
    out->n_levels = P.cartesian ? P.nx + P.ny - 1 : P.nlev_max;
    out->n_self_types = P.nself;
    out->n_nbr_types = P.nnbrt;
    out->general = P.general ? 1 : 0;
    out->n_bdr_attr = P.n_bdr_attr;
    return SMM_OK;
}

int smm_get_quadrature(const smm_problem* prob, double* omega, double* w) {
    if (!prob) return SMM_EINVAL;
    if (omega) std::memcpy(omega, prob->P.omega.data(), sizeof(double) * prob->P.omega.size());
    if (w) std::memcpy(w, prob->P.w.data(), sizeof(double) * prob->P.w.size());
    return SMM_OK;
}

int smm_get_nodes(const smm_problem* prob, double* xy) {
    if (!prob || !xy) return SMM_EINVAL;
    std::memcpy(xy, prob->P.xnode.data(), sizeof(double) * prob->P.xnode.size());
    return SMM_OK;
}

int smm_get_bface_points(const smm_problem* prob, double* xy) {
    if (!prob || !xy) return SMM_EINVAL;
    const Problem& P = prob->P;
    for (int bf = 0; bf < P.nbf; ++bf)
        for (int q = 0; q < P.nq; ++q)
            for (int c = 0; c < 2; ++c)
                xy[((size_t)bf * P.nq + q) * 2 + c] =
                    P.xf[(((size_t)P.bface_K[bf] * 4 + P.bface_f[bf]) * P.nq + q) * 2 + c];
    return SMM_OK;
}

int smm_set_materials(smm_problem* prob, const double* sigma_t, const double* sigma_s) {
    if (!prob || !sigma_t || !sigma_s) return SMM_EINVAL;
    Problem& P = prob->P;
    for (int K = 0; K < P.ne; ++K) {
        if (!(sigma_t[K] > 0.0) || !(sigma_s[K] >= 0.0) || !(sigma_s[K] <= sigma_t[K]) ||
            !std::isfinite(sigma_t[K]))
            return fail(P.ctx, SMM_EINVAL, "need sigma_t > 0 and 0 <= sigma_s <= sigma_t");
    }
    P.sigma_t.assign(sigma_t, sigma_t + P.ne);
    P.sigma_s.assign(sigma_s, sigma_s + P.ne);
    P.have_mat = true;
    P.lhs_ready = false;
    P.cg_ready = false;
    P.rhs_fixed_ready = false;
    P.typed_ready = false;
    P.Pm.clear();
    batch_release_single(prob);
    prob->D.tables_dirty = true;
    prob->D.src_dirty = true;
    return SMM_OK;
}

int smm_set_source(smm_problem* prob, const double* q, int layout) {
    if (!prob || !q) return SMM_EINVAL;
    Problem& P = prob->P;
    size_t cnt;
    if (layout == SMM_SRC_ISO) cnt = (size_t)P.ne * P.n;
    else if (layout == SMM_SRC_ANISO) cnt = (size_t)P.nd * P.ne * P.n;
    else return fail(P.ctx, SMM_EINVAL, "bad source layout");
    for (size_t k = 0; k < cnt; ++k)
        if (!std::isfinite(q[k])) return fail(P.ctx, SMM_EINVAL, "non-finite source");
    P.q.assign(q, q + cnt);
    P.src_layout = layout;
    P.rhs_fixed_ready = false;
    P.typed_ready = false;
    batch_release_single(prob);
    prob->D.src_dirty = true;
    return SMM_OK;
}

int smm_set_inflow(smm_problem* prob, const double* psibar, int layout) {
    if (!prob) return SMM_EINVAL;
    Problem& P = prob->P;
    const size_t full = (size_t)P.nbf * P.nq * P.nd;
    if (layout == SMM_INFLOW_VACUUM) {
        P.psibar.assign(full, 0.0);
    } else if (layout == SMM_INFLOW_ISO_FACE) {
        if (!psibar) return SMM_EINVAL;
        P.psibar.assign(full, 0.0);
        for (int bf = 0; bf < P.nbf; ++bf)
            for (int q = 0; q < P.nq; ++q)
                for (int d = 0; d < P.nd; ++d) P.psibar[((size_t)bf * P.nq + q) * P.nd + d] = psibar[bf];
    } else if (layout == SMM_INFLOW_FULL) {
        if (!psibar) return SMM_EINVAL;
        P.psibar.assign(psibar, psibar + full);
    } else if (layout == SMM_INFLOW_ISO_ATTR) {
        // one isotropic value per boundary attribute: stored as the face-wise
        // isotropic layout it is
        if (!psibar) return SMM_EINVAL;
        P.psibar.assign(full, 0.0);
        for (int bf = 0; bf < P.nbf; ++bf)
            for (int q = 0; q < P.nq; ++q)
                for (int d = 0; d < P.nd; ++d)
                    P.psibar[((size_t)bf * P.nq + q) * P.nd + d] = psibar[P.bface_attr[bf]];
        layout = SMM_INFLOW_ISO_FACE;
    } else {
        return fail(P.ctx, SMM_EINVAL, "bad inflow layout");
    }
    for (double v : P.psibar)
        if (!std::isfinite(v)) return fail(P.ctx, SMM_EINVAL, "non-finite inflow");
    P.inflow_layout = layout;
    P.rhs_fixed_ready = false;
    P.typed_ready = false;
    batch_release_single(prob);
    prob->D.src_dirty = true;
    return SMM_OK;
}

int smm_set_sweep_tiles(smm_problem* prob, int tile_nx, int tile_ny) {
    if (!prob) return SMM_EINVAL;
    Problem& P = prob->P;
    Dev& D = prob->D;
    if (tile_nx < 0 || tile_ny < 0 || (tile_nx == 0) != (tile_ny == 0))
        return fail(P.ctx, SMM_EINVAL, "smm_set_sweep_tiles: tile sizes must both be positive, or both 0");
    if (P.general && tile_nx > 0)
        return fail(P.ctx, SMM_EUNSUPPORTED, "smm_set_sweep_tiles: tiles need a structured mesh");
    if (P.tile_x == tile_nx && P.tile_y == tile_ny) return SMM_OK;
    P.tile_x = tile_nx;
    P.tile_y = tile_ny;
    P.graph_ready = false;
    // the level tables change size: their device copies are rebuilt
    void** tabs[] = {(void**)&D.upflag, (void**)&D.lev_ptr, (void**)&D.lev_elem};
    for (void** t : tabs)
        if (*t) {
            (void)hipFree(*t);
            D.allocs.erase(std::find(D.allocs.begin(), D.allocs.end(), *t));
            *t = nullptr;
        }
    D.gen_sweep_built = false;
    return SMM_OK;
}

// sweep paths 1, 3, 4 and 5 force the per-element kernel (3, 4 and 5 also
// its assembling forms)
static bool per_element_forced(const Dev& D) {
    return D.force_general == 1 || D.force_general >= 3;
}

int smm_set_sweep_path(smm_problem* prob, int force_general) {
    if (!prob) return SMM_EINVAL;
    if (force_general < 0 || force_general > 5) return SMM_EINVAL;
    prob->D.force_general = force_general;
    return SMM_OK;
}

void smm_default_opts(smm_solve_opts* o) {
    if (!o) return;
    o->precision = SMM_FP64;
    o->outer_tol = 1e-10;
    o->max_outer = 200;
    o->inner_tol = 1e-12;
    o->max_inner = 20000;
    o->start = SMM_START_ZERO;
    o->delta_sweeps = 0;
    o->use_graph = 0;
    o->moment_path = 0;
    o->inner_adapt = 0.0;
    o->precond = SMM_PRECOND_BJ;
    o->anderson = 0;
    o->discretization = SMM_DISC_IP;
    o->kappa_scale = 1.0;
    o->start_tol = 0.0;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// host tables and device upload
// ---------------------------------------------------------------------------
// Host tables of the general path (per-element operators); `typed` also
// builds the typed Cartesian blocks instead.
static int ensure_host(smm_problem* pr, bool general = true) {
    Problem& P = pr->P;
    if (!P.have_mat) return fail(P.ctx, SMM_ESTATE, "materials not set");
    if (P.psibar.empty()) P.psibar.assign((size_t)P.nbf * P.nq * P.nd, 0.0);
    if (P.cartesian && P.Pm.empty()) setup_cartesian_operators(P);
    if (general) {
        std::string err;
        int rc = ensure_heavy(P, &err);
        if (rc) return fail(P.ctx, rc, err.empty() ? std::string("geometry setup failed") : err);
        if (!P.lhs_ready) {
            assemble_ip(P);
            assemble_correction_operator(P);
            P.lhs_ready = true;
        }
        if (!P.rhs_fixed_ready) assemble_rhs_fixed(P);
    }
    return SMM_OK;
}

namespace smm {
int ensure_typed(smm_problem* pr) {
    Problem& P = pr->P;
    if (!P.have_mat) return fail(P.ctx, SMM_ESTATE, "materials not set");
    if (!typed_applicable(P)) return fail(P.ctx, SMM_EUNSUPPORTED, "typed path needs a uniform Cartesian mesh, "
                                          "an isotropic source and vacuum or face-wise isotropic inflow");
    int rc = ensure_host(pr, false);
    if (rc) return rc;
    if (!P.typed_ready) {
        std::string err;
        rc = build_typed_blocks(P, err);
        if (rc) return fail(P.ctx, rc, err);
    }
    return SMM_OK;
}
}  // namespace smm

template <typename T>
static int upload(smm_ctx* c, Dev& D, T** dst, const void* src, size_t bytes) {
    if (!*dst) {
        void* ptr = nullptr;
        if (hipMalloc(&ptr, bytes ? bytes : 16) != hipSuccess) return fail(c, SMM_ENOMEM, "hipMalloc failed");
        D.allocs.push_back(ptr);
        *dst = reinterpret_cast<T*>(ptr);
    }
    if (src && bytes)
        if (hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess)
            return fail(c, SMM_EHIP, "hipMemcpy failed");
    return SMM_OK;
}

template <typename T>
static int alloc(smm_ctx* c, Dev& D, T** dst, size_t bytes) {
    return upload(c, D, dst, nullptr, bytes);
}

static std::vector<float> to_f32(const std::vector<double>& v) {
    std::vector<float> o(v.size());
    for (size_t i = 0; i < v.size(); ++i) o[i] = (float)v[i];
    return o;
}

#define UP(dst, vec)                                                              \
    do {                                                                          \
        int rc_ = upload(c, D, &(dst), (vec).data(), sizeof((vec)[0]) * (vec).size()); \
        if (rc_) return rc_;                                                      \
    } while (0)

// Device tables.  Base data (quadrature, Cartesian operator tables, sources,
// work vectors) always; the general sweep's per-element data when
// `gen_sweep`; the per-element moment system when `gen_moment`.
static int ensure_device(smm_problem* pr, bool gen_moment, bool gen_sweep) {
    Problem& P = pr->P;
    Dev& D = pr->D;
    smm_ctx* c = P.ctx;
    if (c->device < 0) return fail(c, SMM_ESTATE, "host-only context");
    if (!P.cartesian || P.tile_x > 0) gen_sweep = true;
    int rc = ensure_host(pr, gen_moment || gen_sweep);
    if (rc) return rc;
    const long L = (long)P.ne * P.n;
    if (!D.built) {
        UP(D.omega, P.omega);
        D.ldw = (P.nd + 3) / 4 * 4;
        std::vector<double> W(16 * (size_t)D.ldw, 0.0);
        for (int d = 0; d < P.nd; ++d) {
            const double w = P.w[d], ox = P.omega[d * 3], oy = P.omega[d * 3 + 1];
            const double rows[8] = {w, w * ox, w * oy, w * ox * ox, w * ox * oy, w * oy * oy, w * std::fabs(ox),
                                    w * std::fabs(oy)};
            for (int r = 0; r < 8; ++r) W[(size_t)r * D.ldw + d] = rows[r];
        }
        std::vector<float> W32 = to_f32(W);
        UP(D.W64, W);
        UP(D.W32, W32);
        std::vector<float> f;
        UP(D.Lf64, P.Lf); f = to_f32(P.Lf); UP(D.Lf32, f);
        UP(D.nbr, P.nbr);
        if (P.general) {
            std::vector<uint8_t> nf(P.nbr_face.size());
            for (size_t k = 0; k < nf.size(); ++k) nf[k] = P.nbr_face[k] < 0 ? 0 : (uint8_t)P.nbr_face[k];
            UP(D.nbr_face, nf);
        }
        if (!P.axis_bdr && P.nbf > 0) {
            std::vector<double> nb2((size_t)P.nbf * P.nq * 2);
            for (int bf = 0; bf < P.nbf; ++bf)
                for (int q = 0; q < P.nq; ++q)
                    for (int k = 0; k < 2; ++k)
                        nb2[((size_t)bf * P.nq + q) * 2 + k] =
                            P.nhat[(((size_t)P.bface_K[bf] * 4 + P.bface_f[bf]) * P.nq + q) * 2 + k];
            UP(D.nhat_b, nb2);
            UP(D.eb0_pt, P.eb0_pt);
            UP(D.w64, P.w);
        }
        UP(D.bface_of, P.bface_of);
        UP(D.bface_K, P.bface_K);
        UP(D.bface_f, P.bface_f);
        const int nd_q = P.nd;  // room for an anisotropic source
        if ((rc = alloc(c, D, &D.S, sizeof(double) * (size_t)nd_q * L))) return rc;
        for (int k = 0; k < 2; ++k)
            if ((rc = alloc(c, D, &D.psi[k], sizeof(double) * (size_t)P.nd * L))) return rc;
        if ((rc = alloc(c, D, &D.mom, sizeof(double) * 8 * L))) return rc;
        if ((rc = alloc(c, D, &D.mom_acc, sizeof(double) * 8 * L))) return rc;
        if ((rc = alloc(c, D, &D.T, sizeof(double) * 3 * L))) return rc;
        if ((rc = alloc(c, D, &D.beta, sizeof(double) * (size_t)std::max(1, P.nbf * P.nq)))) return rc;
        double** vecs[] = {&D.varphi, &D.varphi_prev, &D.x, &D.b, &D.r, &D.z, &D.p, &D.qv};
        for (double** v : vecs)
            if ((rc = alloc(c, D, v, sizeof(double) * L))) return rc;
        const int epb = 256 / P.n;
        D.cg_blocks = (P.ne + epb - 1) / epb;
        if ((rc = alloc(c, D, &D.part, sizeof(double) * 3 * D.cg_blocks))) return rc;
        if ((rc = alloc(c, D, &D.scal, sizeof(double) * 16))) return rc;
        D.r_blocks = (int)std::min<long>(1024, (L + 255) / 256);
        if ((rc = alloc(c, D, &D.rpart, sizeof(double) * 2 * D.r_blocks))) return rc;
        if ((rc = alloc(c, D, &D.rout, sizeof(double) * 2))) return rc;
        D.built = true;
    }
    if (gen_sweep && !D.gen_sweep_built) {
        std::vector<float> f;
        UP(D.Mk64, P.Mk); f = to_f32(P.Mk); UP(D.Mk32, f);
        UP(D.Gx64, P.Gxk); f = to_f32(P.Gxk); UP(D.Gx32, f);
        UP(D.Gy64, P.Gyk); f = to_f32(P.Gyk); UP(D.Gy32, f);
        UP(D.nds64, P.nds); f = to_f32(P.nds); UP(D.nds32, f);
        UP(D.upflag, P.upflag);
        UP(D.lev_ptr, P.lev_ptr);
        UP(D.lev_elem, P.lev_elem);
        D.gen_sweep_built = true;
    }
    if (D.tables_dirty) {
        std::vector<float> f;
        UP(D.st64, P.sigma_t); f = to_f32(P.sigma_t); UP(D.st32, f);
        UP(D.sigma_s, P.sigma_s);
        if (P.cartesian) {
            UP(D.mat, P.mat_of);
            // tables may grow when the material count changes: reallocate
            auto reup = [&](void** dst64, void** dst32, const std::vector<double>& v) -> int {
                if (*dst64) { (void)hipFree(*dst64); D.allocs.erase(std::find(D.allocs.begin(), D.allocs.end(), *dst64)); *dst64 = nullptr; }
                if (*dst32) { (void)hipFree(*dst32); D.allocs.erase(std::find(D.allocs.begin(), D.allocs.end(), *dst32)); *dst32 = nullptr; }
                int r1 = upload(c, D, dst64, v.data(), sizeof(double) * v.size());
                if (r1) return r1;
                std::vector<float> g = to_f32(v);
                return upload(c, D, dst32, g.data(), sizeof(float) * g.size());
            };
            if ((rc = reup(&D.Pm64, &D.Pm32, P.Pm))) return rc;
            if ((rc = reup(&D.Px64, &D.Px32, P.Px))) return rc;
            if ((rc = reup(&D.Py64, &D.Py32, P.Py))) return rc;
        }
        D.tables_dirty = false;
        D.gen_dirty = true;
        D.inv_ready[0] = D.inv_ready[1] = false;   // the element operators hold sigma_t
    }
    if (D.src_dirty) {
        UP(D.q, P.q);
        // inflow: [nd][nbf][nq] for the general kernel, traces for the cartesian kernel
        std::vector<double> pb((size_t)P.nd * P.nbf * P.nq);
        for (int bf = 0; bf < P.nbf; ++bf)
            for (int q = 0; q < P.nq; ++q)
                for (int d = 0; d < P.nd; ++d)
                    pb[((size_t)d * P.nbf + bf) * P.nq + q] = P.psibar[((size_t)bf * P.nq + q) * P.nd + d];
        std::vector<float> f = to_f32(pb);
        UP(D.pbar64, pb);
        UP(D.pbar32, f);
        if (P.cartesian) {
            std::vector<double> bx, by;
            cartesian_boundary_traces(P, bx, by);
            UP(D.bx64, bx); f = to_f32(bx); UP(D.bx32, f);
            UP(D.by64, by); f = to_f32(by); UP(D.by32, f);
        }
        D.src_dirty = false;
        D.gen_dirty = true;
        D.inv_ready[0] = D.inv_ready[1] = false;   // the element operators hold the inflow
    }
    if (gen_moment && D.gen_dirty) {
        UP(D.bsr_col, P.bsr_col);
        UP(D.bsr_val, P.bsr_val);
        UP(D.bjac, P.bjac_inv);
        UP(D.corr, P.corr_val);
        if (P.nbf > 0) UP(D.beta_op, P.beta_op);
        UP(D.bfix, P.b_fixed);
        D.gen_dirty = false;
    }
    return SMM_OK;
}

// ---------------------------------------------------------------------------
// kernels of one outer iteration
// ---------------------------------------------------------------------------
// arguments of the per-element sweep with the tables of one precision
static GenSweepArgs gen_args(smm_problem* pr, bool fp64) {
    Problem& P = pr->P;
    Dev& D = pr->D;
    GenSweepArgs a{};
    a.ne = P.ne; a.nd = P.nd; a.nb = P.nb; a.nq = P.nq; a.nbf = P.nbf; a.nlev = P.nlev_max;
    a.ntiles = P.ntiles;
    a.maxw = P.lev_wmax;
    a.Mk = fp64 ? D.Mk64 : D.Mk32;
    a.Gx = fp64 ? D.Gx64 : D.Gx32;
    a.Gy = fp64 ? D.Gy64 : D.Gy32;
    a.nds = fp64 ? D.nds64 : D.nds32;
    a.Lf = fp64 ? D.Lf64 : D.Lf32;
    a.sigma_t = fp64 ? D.st64 : D.st32;
    a.nbr = D.nbr;
    a.nbr_face = P.general ? D.nbr_face : nullptr;
    a.bface_of = D.bface_of;
    a.upflag = D.upflag;
    a.lev_ptr = D.lev_ptr;
    a.lev_elem = D.lev_elem;
    a.omega = D.omega;
    return a;
}

// Stored element operators of the per-element sweep in one precision: built
// from the FP64 tables on first use after a change of sigma_t.  *use stays
// false (the sweep then assembles and eliminates per element) when they would
// take more than a quarter of the free device memory, or inside the
// no-allocation entry point before their memory exists.
static int ensure_inv(smm_problem* pr, bool fp64, bool* use) {
    Problem& P = pr->P;
    Dev& D = pr->D;
    smm_ctx* c = P.ctx;
    const int k = fp64 ? 1 : 0;
    *use = false;
    if (D.inv_ready[k]) {
        *use = true;
        return SMM_OK;
    }
    const size_t es = fp64 ? sizeof(double) : sizeof(float);
    const size_t pairs = (size_t)P.nd * P.ne;
    const size_t bytes_A = es * pairs * P.n * P.n, bytes_C = es * pairs * P.n, bytes_G = es * pairs * 4 * P.nb * P.n;
    if (!D.inv_A[k]) {
        if (D.noalloc_active) return SMM_OK;
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess || bytes_A + bytes_C + bytes_G + pairs > fr / 4) return SMM_OK;
        int rc = alloc(c, D, &D.inv_A[k], bytes_A);
        if (!rc) rc = alloc(c, D, &D.inv_C[k], bytes_C);
        if (!rc) rc = alloc(c, D, &D.inv_G[k], bytes_G);
        if (!rc && !D.inv_mask) rc = alloc(c, D, &D.inv_mask, pairs);
        if (rc) return rc;
    }
    GenSweepArgs a = gen_args(pr, true);
    a.psibar = P.inflow_layout != SMM_INFLOW_VACUUM ? D.pbar64 : nullptr;
    const hipError_t e = launch_gen_inv_setup(fp64, a, D.inv_A[k], D.inv_C[k], D.inv_G[k], D.inv_mask, c->stream);
    if (e != hipSuccess) return fail(c, SMM_EHIP, std::string("element operator set-up: ") + hipGetErrorString(e));
    D.inv_ready[k] = true;
    *use = true;
    return SMM_OK;
}

static int run_sweep(smm_problem* pr, bool fp64, const void* S, int s_aniso, const void* psi_lag, void* psi_out,
                     bool with_inflow) {
    Problem& P = pr->P;
    Dev& D = pr->D;
    smm_ctx* c = P.ctx;
    hipError_t e;
    if (P.cartesian && !per_element_forced(D) && P.tile_x == 0) {
        CartSweepArgs a{};
        a.nx = P.nx; a.ny = P.ny; a.nd = P.nd; a.nb = P.nb; a.nmat = P.nmat;
        a.s_aniso = s_aniso;
        a.S = S;
        a.Pm = fp64 ? D.Pm64 : D.Pm32;
        a.Px = fp64 ? D.Px64 : D.Px32;
        a.Py = fp64 ? D.Py64 : D.Py32;
        a.mat = D.mat;
        a.omega = D.omega;
        a.bx = with_inflow && P.inflow_layout != SMM_INFLOW_VACUUM ? (fp64 ? D.bx64 : D.bx32) : nullptr;
        a.by = with_inflow && P.inflow_layout != SMM_INFLOW_VACUUM ? (fp64 ? D.by64 : D.by32) : nullptr;
        a.psi = psi_out;
        a.variant = D.force_general == 2 ? 1 : 0;
        e = launch_sweep_cart(fp64, a, c->stream);
    } else {
        GenSweepArgs a = gen_args(pr, fp64);
        a.wave_solve = D.force_general == 3 ? 1 : (D.force_general == 4 ? 2 : 0);
        a.s_aniso = s_aniso;
        a.S = S;
        a.psibar = with_inflow && P.inflow_layout != SMM_INFLOW_VACUUM ? (fp64 ? D.pbar64 : D.pbar32) : nullptr;
        a.psi_lag = psi_lag;
        a.psi = psi_out;
        if (D.force_general <= 1) {
            bool use = false;
            const int rc = ensure_inv(pr, fp64, &use);
            if (rc) return rc;
            if (use) {
                const int k = fp64 ? 1 : 0;
                a.invA = D.inv_A[k];
                a.invC = D.inv_C[k];
                a.invG = D.inv_G[k];
                a.inmask = D.inv_mask;
            }
        }
        e = launch_sweep_general(fp64, a, c->stream);
    }
    if (e != hipSuccess) return fail(c, SMM_EHIP, std::string("sweep launch: ") + hipGetErrorString(e));
    return SMM_OK;
}

static CgState cg_state(smm_problem* pr) {
    Problem& P = pr->P;
    Dev& D = pr->D;
    CgState s{};
    s.ne = P.ne; s.n = P.n;
    s.col = D.bsr_col; s.A = D.bsr_val; s.Dinv = D.bjac; s.b = D.b;
    s.x = D.x; s.r = D.r; s.z = D.z; s.p = D.p; s.q = D.qv;
    s.part = D.part; s.scal = D.scal; s.nblocks = D.cg_blocks;
    return s;
}

// Solve the IP system for b (already in D.b) starting from D.x.  Returns the
// CG iteration count in *its.
// Continuous (CG) moment system on the device: host assembly on first use or
// after a material change, then upload.
static int ensure_cg(smm_problem* pr) {
    if (pr->P.general) return fail(pr->P.ctx, SMM_EUNSUPPORTED, "the CG moment system needs a structured mesh");
    Problem& P = pr->P;
    Dev& D = pr->D;
    smm_ctx* c = P.ctx;
    if (!P.cg_ready) {
        assemble_cg(P);
        D.cg_dirty = true;
        D.cg_mg_dirty = true;
    }
    if (D.cg_twolevel && D.cg_mg_dirty) {
        MGHost M;
        std::string err;
        const int rc = build_mg_cg(P, M, err);
        if (rc) return fail(c, rc, "two-level preconditioner of the CG system: " + err);
        if ((int)M.lev.size() > CGS_MG_MAXLEV || P.p + 1 > 8)
            return fail(c, SMM_EUNSUPPORTED, "two-level preconditioner of the CG system: too many levels");
        D.cg_mg_nlev = (int)M.lev.size();
        for (int l = 0; l < D.cg_mg_nlev; ++l) {
            const size_t nv = (size_t)M.lev[l].nvx * M.lev[l].nvy;
            D.cg_mg_nvx[l] = M.lev[l].nvx;
            D.cg_mg_nvy[l] = M.lev[l].nvy;
            UP(D.cg_mg_A[l], M.lev[l].A);
            double** vecs[] = {&D.cg_mg_x[l], &D.cg_mg_t[l], &D.cg_mg_b[l]};
            for (double** v : vecs) {
                const int rc2 = alloc(c, D, v, sizeof(double) * nv);
                if (rc2) return rc2;
            }
        }
        UP(D.cg_mg_cinv, M.cinv);
        for (size_t k = 0; k < M.gll.size() && k < 8; ++k) D.cg_mg_gll[k] = M.gll[k];
        D.cg_mg_dirty = false;
    }
    if (D.cg_dirty) {
        UP(D.cg_rowptr, P.cg_rowptr);
        UP(D.cg_col, P.cg_col);
        UP(D.cg_val, P.cg_val);
        UP(D.cg_dinv, P.cg_dinv);
        UP(D.cg_tab, P.cg_tab);
        UP(D.cg_map, P.cg_map);
        const size_t nc = (size_t)P.cg_nc;
        double** vecs[] = {&D.cg_b, &D.cg_x, &D.cg_r, &D.cg_z, &D.cg_p, &D.cg_q};
        int rc;
        for (double** v : vecs)
            if ((rc = alloc(c, D, v, sizeof(double) * nc))) return rc;
        const size_t vb = (nc + 255) / 256, sb = (nc + CGS_SPMV_ROWS - 1) / CGS_SPMV_ROWS;
        if ((rc = alloc(c, D, &D.cg_part, sizeof(double) * (sb + 3 * vb)))) return rc;
        if ((rc = alloc(c, D, &D.cg_scal, sizeof(double) * 16))) return rc;
        D.cg_dirty = false;
    }
    return SMM_OK;
}

static CgsArgs cgs_args(smm_problem* pr) {
    Problem& P = pr->P;
    Dev& D = pr->D;
    CgsArgs a{};
    a.nc = P.cg_nc;
    a.L = (long)P.ne * P.n;
    a.rowptr = D.cg_rowptr; a.col = D.cg_col; a.val = D.cg_val; a.dinv = D.cg_dinv;
    a.tab = D.cg_tab; a.map = D.cg_map;
    a.b = D.cg_b; a.x = D.cg_x; a.r = D.cg_r; a.z = D.cg_z; a.p = D.cg_p; a.q = D.cg_q;
    a.part = D.cg_part; a.scal = D.cg_scal;
    a.vblocks = (P.cg_nc + 255) / 256;
    a.sblocks = (P.cg_nc + CGS_SPMV_ROWS - 1) / CGS_SPMV_ROWS;
    a.mg = D.cg_twolevel ? 1 : 0;
    a.nx = P.nx;
    a.ny = P.ny;
    a.order = P.p;
    for (int k = 0; k < 8; ++k) a.gll[k] = D.cg_mg_gll[k];
    if (a.mg) {
        a.rv = D.cg_mg_b[0];
        a.xv = D.cg_mg_nlev > 1 ? D.cg_mg_t[0] : D.cg_mg_x[0];   // the V-cycle ends in t above the coarsest level
    }
    return a;
}

static CgsMG cgs_mg(smm_problem* pr) {
    Dev& D = pr->D;
    CgsMG m{};
    m.nlev = D.cg_mg_nlev;
    for (int l = 0; l < m.nlev; ++l) {
        m.nvx[l] = D.cg_mg_nvx[l];
        m.nvy[l] = D.cg_mg_nvy[l];
        m.A[l] = D.cg_mg_A[l];
        m.x[l] = D.cg_mg_x[l];
        m.t[l] = D.cg_mg_t[l];
        m.b[l] = D.cg_mg_b[l];
    }
    m.cinv = D.cg_mg_cinv;
    m.omega = 2.0 / 3.0;
    return m;
}

// The CG moment solve: restrict the DG right-hand side D.b to V_p, start from
// the DG iterate in D.x (continuous after the first CG solve, so its node
// values are exact), Jacobi-PCG, and return the DG values P_c c in D.x.
static int cg_moment_solve(smm_problem* pr, double tol, int max_inner, int* its, bool graph, bool* conv = nullptr) {
    Dev& D = pr->D;
    smm_ctx* c = pr->P.ctx;
    const CgsArgs a = cgs_args(pr);
    const CgsMG m = cgs_mg(pr);
    HIPCHK(c, cgs_gather(a, D.b, c->stream));
    HIPCHK(c, cgs_pick(a, D.x, c->stream));
    HIPCHK(c, cgs_start(a, m, tol, c->stream));
    double sc[8];
    int chunk = 4, done = 0;
    while (true) {
        HIPCHK(c, hipMemcpyAsync(sc, D.cg_scal, sizeof(double) * 8, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        done = (int)sc[5];
        if (sc[6] == 2.0) return fail(c, SMM_ENAN, "non-finite values in the moment solve (continuous system)");
        if (sc[6] != 0.0) return fail(c, SMM_EBREAKDOWN, "CG breakdown (continuous moment system)");
        if (sc[4] != 0.0 || done >= max_inner) break;
        const int k = std::min(chunk, max_inner - done);
        if (graph) {
            // capture the chunk of k iterations once on a private stream
            // (kernel nodes only), then replay it on the context's stream
            hipGraphExec_t ge = nullptr;
            const int key = 2 * k + a.mg;
            for (auto& e : D.cg_graphs)
                if (e.first == key) ge = e.second;
            if (!ge) {
                if (!D.cg_cap) HIPCHK(c, hipStreamCreateWithFlags(&D.cg_cap, hipStreamNonBlocking));
                hipGraph_t g = nullptr;
                HIPCHK(c, hipStreamBeginCapture(D.cg_cap, hipStreamCaptureModeRelaxed));
                const hipError_t e1 = cgs_iterations(a, m, k, D.cg_cap);
                const hipError_t e2 = hipStreamEndCapture(D.cg_cap, &g);
                if (e1 != hipSuccess || e2 != hipSuccess) {
                    if (g) (void)hipGraphDestroy(g);
                    return fail(c, SMM_EHIP, "CG graph capture failed");
                }
                const hipError_t e3 = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (e3 != hipSuccess) return fail(c, SMM_EHIP, "CG graph instantiation failed");
                D.cg_graphs.emplace_back(key, ge);
            }
            HIPCHK(c, hipGraphLaunch(ge, c->stream));
        } else {
            HIPCHK(c, cgs_iterations(a, m, k, c->stream));
        }
        chunk = std::min(chunk * 2, 64);
    }
    HIPCHK(c, cgs_scatter(a, D.x, c->stream));
    *its = done;
    if (conv) *conv = sc[4] != 0.0;
    return SMM_OK;
}

static int moment_solve(smm_problem* pr, double tol, int max_inner, int* its, bool* conv = nullptr) {
    Problem& P = pr->P;
    Dev& D = pr->D;
    smm_ctx* c = P.ctx;
    CgState s = cg_state(pr);
    HIPCHK(c, cg_start(s, tol, c->stream));
    int done_its = 0;
    double sc[8];
    int chunk = 4;
    while (true) {
        HIPCHK(c, hipMemcpyAsync(sc, D.scal, sizeof(double) * 8, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        done_its = (int)sc[5];
        if (sc[6] == 2.0) return fail(c, SMM_ENAN, "non-finite values in the moment solve");
        if (sc[6] != 0.0) return fail(c, SMM_EBREAKDOWN, "CG breakdown");
        if (sc[4] != 0.0) break;
        if (done_its >= max_inner) break;
        const int k = std::min(chunk, max_inner - done_its);
        HIPCHK(c, cg_iterations(s, k, tol, c->stream));
        chunk = std::min(chunk * 2, 64);
    }
    *its = done_its;
    if (conv) *conv = sc[4] != 0.0 && sc[6] == 0.0;
    return SMM_OK;
}

// One evaluation of G from D.varphi into D.x (b, closures, moments updated).
// psi_cur / psi_prev are sweep buffers; delta mode sweeps sigma_s/(4pi)(varphi - varphi_prev).
static int eval_G(smm_problem* pr, bool fp64, bool delta, bool first, int cur, double inner_tol, int max_inner,
                  int* cg_its, bool cgdisc = false, bool graph = false, bool* conv = nullptr, bool timed = false) {
    Problem& P = pr->P;
    Dev& D = pr->D;
    smm_ctx* c = P.ctx;
    const long L = (long)P.ne * P.n;
    const bool aniso = P.src_layout == SMM_SRC_ANISO;
    const int nd_q = aniso ? P.nd : 1;
    int rc;
    if (timed) HIPCHK(c, hipEventRecord(D.ev[0], c->stream));
    // scattering source (a1)
    if (!delta || first) {
        HIPCHK(c, launch_source(fp64, P.ne, P.n, nd_q, D.sigma_s, D.varphi, nullptr, D.q, D.S, c->stream));
    } else {
        HIPCHK(c, launch_source(fp64, P.ne, P.n, 1, D.sigma_s, D.varphi, D.varphi_prev, nullptr, D.S, c->stream));
    }
    const bool s_aniso = aniso && (!delta || first);
    // sweep (a2): the previous sweep serves as the lagged input on curved meshes
    void* out = D.psi[cur];
    const void* lag = first ? nullptr : D.psi[cur ^ 1];
    if ((rc = run_sweep(pr, fp64, D.S, s_aniso ? 1 : 0, lag, out, !delta || first))) return rc;
    if (timed) HIPCHK(c, hipEventRecord(D.ev[1], c->stream));
    // moments (a3)
    HIPCHK(c, launch_moments(fp64, out, P.nd, L, fp64 ? D.W64 : D.W32, D.ldw, D.mom, c->stream));
    const double* mom = D.mom;
    if (delta) {
        if (first) HIPCHK(c, hipMemsetAsync(D.mom_acc, 0, sizeof(double) * 8 * L, c->stream));
        HIPCHK(c, launch_axpy_mom(8 * L, D.mom, D.mom_acc, c->stream));
        mom = D.mom_acc;
    }
    D.last_mom = mom;
    // closures (a4) and right-hand side (a5)
    HIPCHK(c, launch_closures(P.ne, P.n, P.nb, P.nq, P.axis_bdr ? P.nbf : 0, mom, D.bface_K, D.bface_f,
                              (const double*)D.Lf64, P.eb0x, P.eb0y, D.T, D.beta, c->stream));
    if (!P.axis_bdr)   // beta from psi itself, accumulated over delta sweeps like the moments
        HIPCHK(c, launch_beta_general(fp64, P.nd, P.ne, P.n, P.nb, P.nq, P.nbf, out, D.omega, D.w64, D.bface_K,
                                      D.bface_f, D.nhat_b, D.eb0_pt, (const double*)D.Lf64, delta && !first,
                                      D.beta, c->stream));
    HIPCHK(c, launch_rhs(P.ne, P.n, P.nq, D.bfix, D.bsr_col, D.corr, D.T, D.bface_of, D.beta_op, D.beta, D.b,
                         c->stream));
    // moment solve (a6), warm-started from the current iterate
    HIPCHK(c, hipMemcpyAsync(D.x, D.varphi, sizeof(double) * L, hipMemcpyDeviceToDevice, c->stream));
    if (timed) HIPCHK(c, hipEventRecord(D.ev[2], c->stream));
    rc = cgdisc ? cg_moment_solve(pr, inner_tol, max_inner, cg_its, graph, conv)
                : moment_solve(pr, inner_tol, max_inner, cg_its, conv);
    if (!rc && timed) HIPCHK(c, hipEventRecord(D.ev[3], c->stream));
    return rc;
}

extern "C" {

int smm_solve(smm_problem* prob, const smm_solve_opts* opts, const double* varphi0, smm_solve_info* info) {
    if (!prob) return SMM_EINVAL;
    smm_solve_opts o;
    smm_default_opts(&o);
    if (opts) o = *opts;
    Problem& P = prob->P;
    Dev& D = prob->D;
    smm_ctx* c = P.ctx;
    if (c->device < 0) return fail(c, SMM_ESTATE, "host-only context");
    if (!P.have_mat) return fail(c, SMM_ESTATE, "materials not set");
    if (!(o.start_tol >= 0)) return fail(c, SMM_EINVAL, "start_tol must be >= 0");
    if (o.discretization != SMM_DISC_IP && o.discretization != SMM_DISC_CG)
        return fail(c, SMM_EINVAL, "smm_solve: discretization must be SMM_DISC_IP or SMM_DISC_CG");
    const bool cgdisc = o.discretization == SMM_DISC_CG;
    if (cgdisc && o.precond != SMM_PRECOND_BJ && o.precond != SMM_PRECOND_TWOLEVEL)
        return fail(c, SMM_EINVAL, "smm_solve: unknown preconditioner");
    if (cgdisc) D.cg_twolevel = o.precond == SMM_PRECOND_TWOLEVEL;
    if (cgdisc && P.general)
        return fail(c, SMM_EUNSUPPORTED, "smm_solve: the CG moment system needs a structured mesh");
    if (cgdisc && o.anderson != 0)
        return fail(c, SMM_EUNSUPPORTED, "smm_solve: Anderson mixing runs on the typed path, IP discretisation only");
    if (o.anderson != 0 && !(o.moment_path == 0 && typed_applicable(P) && !per_element_forced(D) && P.tile_x == 0))
        return fail(c, SMM_EUNSUPPORTED, "smm_solve: Anderson mixing needs the typed (batched) path");
    if (o.start < SMM_START_ZERO || o.start > SMM_START_LEARNED)
        return fail(c, SMM_EINVAL, "smm_solve: unknown start mode");
    if (!(o.kappa_scale >= 0.0) || !std::isfinite(o.kappa_scale))
        return fail(c, SMM_EINVAL, "smm_solve: kappa_scale must be finite and >= 0");
    if (o.kappa_scale != P.kappa_scale) {
        // a new penalty: the moment system is assembled again
        P.kappa_scale = o.kappa_scale;
        P.lhs_ready = false;
        P.typed_ready = false;
        batch_release_single(prob);
        D.gen_dirty = true;
    }
    const bool typed = !cgdisc && o.moment_path == 0 && typed_applicable(P) && !per_element_forced(D) && P.tile_x == 0;
    if (o.start == SMM_START_LEARNED && !typed)
        return fail(c, SMM_EUNSUPPORTED, "smm_solve: the learned start needs the typed path (uniform Cartesian mesh, "
                                         "isotropic source, IP moment system)");
    if (typed) {
        const int r = batch_solve_single(prob, o, varphi0, info);
        D.last_typed = (r == SMM_OK || r == SMM_ENOCONV);
        batch_history_single(prob, D.hist_r, D.hist_cg);
        return r;
    }
    D.hist_r.clear();
    D.hist_cg.clear();
    D.last_typed = false;
    auto t0 = std::chrono::steady_clock::now();
    int rc = ensure_device(prob, true, per_element_forced(D));
    if (rc) return rc;
    if (cgdisc && (rc = ensure_cg(prob))) return rc;
    const long L = (long)P.ne * P.n;
    const bool fp64 = o.precision == SMM_FP64;
    const bool delta = o.delta_sweeps != 0;
    int its = 0;
    if (o.start == SMM_START_GIVEN) {
        if (!varphi0) return fail(c, SMM_EINVAL, "varphi0 required");
        HIPCHK(c, hipMemcpyAsync(D.varphi, varphi0, sizeof(double) * L, hipMemcpyHostToDevice, c->stream));
    } else if (o.start == SMM_START_DIFFUSION) {
        HIPCHK(c, hipMemcpyAsync(D.b, D.bfix, sizeof(double) * L, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(c, hipMemsetAsync(D.x, 0, sizeof(double) * L, c->stream));
        rc = cgdisc ? cg_moment_solve(prob, start_tol(o), o.max_inner, &its, o.use_graph != 0)
                    : moment_solve(prob, start_tol(o), o.max_inner, &its);
        if (rc) return rc;
        HIPCHK(c, hipMemcpyAsync(D.varphi, D.x, sizeof(double) * L, hipMemcpyDeviceToDevice, c->stream));
    } else {
        HIPCHK(c, hipMemsetAsync(D.varphi, 0, sizeof(double) * L, c->stream));
    }
    HIPCHK(c, hipMemsetAsync(D.varphi_prev, 0, sizeof(double) * L, c->stream));
    auto t1 = std::chrono::steady_clock::now();   // tables and start ready
    for (auto& e : D.ev)
        if (!e) HIPCHK(c, hipEventCreate(&e));
    D.phase_ms[0] = D.phase_ms[1] = D.phase_ms[2] = D.phase_ms[3] = 0.0;
    int cg_total = 0, cg_max = 0;
    double r = 0, rabs = 0;
    int it = 0;
    int status = SMM_ENOCONV;
    double r_prev = 1.0;
    for (it = 1; it <= o.max_outer; ++it) {
        int cgi = 0;
        const double tol_k = o.inner_adapt > 0 ? std::max(o.inner_tol, o.inner_adapt * r_prev) : o.inner_tol;
        bool inner_ok = true;
        if ((rc = eval_G(prob, fp64, delta, it == 1, it & 1, tol_k, o.max_inner, &cgi, cgdisc, o.use_graph != 0,
                         &inner_ok, true)))
            return rc;
        cg_total += cgi;
        cg_max = std::max(cg_max, cgi);
        // residual (a7)
        HIPCHK(c, launch_residual(L, D.x, D.varphi, D.rpart, D.r_blocks, D.rout, c->stream));
        double ro[2];
        HIPCHK(c, hipMemcpyAsync(ro, D.rout, sizeof(double) * 2, hipMemcpyDeviceToHost, c->stream));
        // shift iterates: varphi_prev <- varphi, varphi <- x
        std::swap(D.varphi_prev, D.varphi);
        std::swap(D.varphi, D.x);
        HIPCHK(c, hipEventRecord(D.ev[4], c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (int ph = 0; ph < 4; ++ph) {
            float ms = 0;
            HIPCHK(c, hipEventElapsedTime(&ms, D.ev[ph], D.ev[ph + 1]));
            D.phase_ms[ph] += ms;
        }
        rabs = ro[0];
        r = ro[1] > 0 ? ro[0] / ro[1] : (ro[0] == 0 ? 0.0 : INFINITY);
        D.hist_r.push_back(r);
        D.hist_cg.push_back(cgi);
        if (!std::isfinite(r) || !std::isfinite(rabs)) { status = SMM_ENAN; break; }
        // with adaptive inner tolerances, convergence counts only from a
        // moment solve as tight as the target residual asks for (a looser
        // solve can stop before moving X); else one more, tighter, iteration
        const double tight = o.inner_adapt > 0 ? std::max(o.inner_tol, o.inner_adapt * o.outer_tol) : o.inner_tol;
        if (r < o.outer_tol && tol_k <= tight && inner_ok) { status = SMM_OK; break; }
        r_prev = r;
    }
    D.last_varphi = D.varphi;
    if (it > o.max_outer) it = o.max_outer;
    D.have_outputs = true;
    auto t2 = std::chrono::steady_clock::now();
    if (info) {
        info->iterations = it;
        info->residual = r;
        info->residual_abs = rabs;
        info->cg_iterations_total = cg_total;
        info->cg_iterations_max = cg_max;
        info->t_total_ms = std::chrono::duration<double, std::milli>(t2 - t0).count();
        info->t_setup_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        info->t_sweep_ms = D.phase_ms[0];
        info->t_moments_ms = D.phase_ms[1];
        info->t_cg_ms = D.phase_ms[2];
        info->t_residual_ms = D.phase_ms[3];
    }
    if (status == SMM_ENAN) return fail(c, SMM_ENAN, "non-finite residual");
    if (status == SMM_ENOCONV) return fail(c, SMM_ENOCONV, "max_outer reached");
    return SMM_OK;
}

int smm_solve_history(const smm_problem* prob, int max_len, double* residual, int* cg_iterations, int* len) {
    if (!prob || !len || max_len < 0) return SMM_EINVAL;
    const Dev& D = prob->D;
    *len = (int)D.hist_r.size();
    const int k = std::min(max_len, *len);
    if (residual) std::copy(D.hist_r.begin(), D.hist_r.begin() + k, residual);
    if (cg_iterations) std::copy(D.hist_cg.begin(), D.hist_cg.begin() + k, cg_iterations);
    return SMM_OK;
}

int smm_get_outputs(smm_problem* prob, double* varphi, double* phi, double* J, double* T, double* beta,
                    int on_device) {
    if (!prob) return SMM_EINVAL;
    Problem& P = prob->P;
    Dev& D = prob->D;
    smm_ctx* c = P.ctx;
    if (D.last_typed) return batch_outputs_single(prob, varphi, phi, J, T, beta, on_device);
    if (!D.have_outputs || !D.last_mom) return fail(c, SMM_ESTATE, "no solve has run");
    const long L = (long)P.ne * P.n;
    const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (varphi && D.last_varphi)
        HIPCHK(c, hipMemcpyAsync(varphi, D.last_varphi, sizeof(double) * L, k, c->stream));
    if (phi) HIPCHK(c, hipMemcpyAsync(phi, D.last_mom, sizeof(double) * L, k, c->stream));
    if (J) HIPCHK(c, hipMemcpyAsync(J, D.last_mom + L, sizeof(double) * 2 * L, k, c->stream));
    if (T) HIPCHK(c, hipMemcpyAsync(T, D.T, sizeof(double) * 3 * L, k, c->stream));
    if (beta && P.nbf > 0)
        HIPCHK(c, hipMemcpyAsync(beta, D.beta, sizeof(double) * P.nbf * P.nq, k, c->stream));
    if (!on_device) HIPCHK(c, hipStreamSynchronize(c->stream));
    return SMM_OK;
}

int smm_apply_sweep(smm_problem* prob, int precision, const void* S, int s_layout, const void* psi_lag,
                    void* psi_out, int with_inflow) {
    if (!prob || !S || !psi_out) return SMM_EINVAL;
    if (precision != SMM_FP64 && precision != SMM_FP32_SWEEP) return SMM_EINVAL;
    if (s_layout != SMM_SRC_ISO && s_layout != SMM_SRC_ANISO) return SMM_EINVAL;
    int rc = ensure_device(prob, false, per_element_forced(prob->D));
    if (rc) return rc;
    return run_sweep(prob, precision == SMM_FP64, S, s_layout == SMM_SRC_ANISO ? 1 : 0, psi_lag, psi_out,
                     with_inflow != 0);
}

int smm_apply_moments(smm_problem* prob, int precision, const void* psi, double* mom) {
    if (!prob || !psi || !mom) return SMM_EINVAL;
    if (precision != SMM_FP64 && precision != SMM_FP32_SWEEP) return SMM_EINVAL;
    int rc = ensure_device(prob, false, false);
    if (rc) return rc;
    Problem& P = prob->P;
    Dev& D = prob->D;
    const bool fp64 = precision == SMM_FP64;
    HIPCHK(P.ctx, launch_moments(fp64, psi, P.nd, (long)P.ne * P.n, fp64 ? D.W64 : D.W32, D.ldw, mom,
                                 P.ctx->stream));
    return SMM_OK;
}

int smm_apply_G(smm_problem* prob, int precision, const double* varphi_in, double* varphi_out, double inner_tol,
                int max_inner) {
    if (!prob || !varphi_in || !varphi_out) return SMM_EINVAL;
    int rc = ensure_device(prob, true, per_element_forced(prob->D));
    if (rc) return rc;
    Problem& P = prob->P;
    Dev& D = prob->D;
    smm_ctx* c = P.ctx;
    const long L = (long)P.ne * P.n;
    HIPCHK(c, hipMemcpyAsync(D.varphi, varphi_in, sizeof(double) * L, hipMemcpyDeviceToDevice, c->stream));
    int its = 0;
    if ((rc = eval_G(prob, precision == SMM_FP64, false, true, 0, inner_tol, max_inner, &its))) return rc;
    HIPCHK(c, hipMemcpyAsync(varphi_out, D.x, sizeof(double) * L, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    D.have_outputs = true;
    D.last_varphi = D.x;
    D.last_typed = false;
    return SMM_OK;
}

int smm_apply_G_noalloc(smm_problem* prob, int precision, const double* varphi_in, double* varphi_out,
                        double inner_tol, int max_inner) {
    if (!prob || !varphi_in || !varphi_out) return SMM_EINVAL;
    Problem& P = prob->P;
    Dev& D = prob->D;
    smm_ctx* c = P.ctx;
    if (precision != SMM_FP64 && precision != SMM_FP32_SWEEP)
        return fail(c, SMM_EINVAL, "smm_apply_G_noalloc: unknown precision");
    if (c->device < 0) return fail(c, SMM_ESTATE, "host-only context");
    if (c->device >= kMaxDevices) return fail(c, SMM_EUNSUPPORTED, "smm_apply_G_noalloc: device index too large");
    // every table must already be on the device (this call uploads nothing)
    const bool gen_sweep = !P.cartesian || P.tile_x > 0 || per_element_forced(D);
    if (!D.built || D.tables_dirty || D.src_dirty || D.gen_dirty || !P.lhs_ready || !P.rhs_fixed_ready ||
        (gen_sweep && !D.gen_sweep_built) || !P.graph_ready)
        return fail(c, SMM_ESTATE, "smm_apply_G_noalloc: the problem's tables are not on the device; call smm_apply_G "
                                   "once after the last change of materials, source or inflow");
    void* base;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        base = g_scratch_ptr[c->device];
    }
    if (!base) return fail(c, SMM_ESTATE, "smm_apply_G_noalloc: no scratch address for this device");
    // carve the work vectors of one evaluation of G out of the array
    const size_t L = (size_t)P.ne * P.n;
    const size_t nd_q = P.src_layout == SMM_SRC_ANISO ? (size_t)P.nd : 1;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += (bytes + 255) / 256 * 256;
        return static_cast<unsigned char*>(base) + at;
    };
    Dev saved = D;
    struct Restore {
        Dev& d;
        Dev& s;
        ~Restore() {
            d.varphi = s.varphi; d.S = s.S; d.psi[0] = s.psi[0]; d.mom = s.mom; d.T = s.T; d.beta = s.beta;
            d.x = s.x; d.b = s.b; d.r = s.r; d.z = s.z; d.p = s.p; d.qv = s.qv; d.part = s.part; d.scal = s.scal;
            d.last_mom = s.last_mom; d.last_varphi = s.last_varphi;
            d.noalloc_active = false;
        }
    } restore{D, saved};
    D.noalloc_active = true;
    D.varphi = reinterpret_cast<double*>(take(sizeof(double) * L));
    D.S = take(sizeof(double) * nd_q * L);
    D.psi[0] = take(sizeof(double) * (size_t)P.nd * L);
    D.mom = reinterpret_cast<double*>(take(sizeof(double) * 8 * L));
    D.T = reinterpret_cast<double*>(take(sizeof(double) * 3 * L));
    D.beta = reinterpret_cast<double*>(take(sizeof(double) * (size_t)std::max(1, P.nbf * P.nq)));
    double** vecs[] = {&D.x, &D.b, &D.r, &D.z, &D.p, &D.qv};
    for (double** v : vecs) *v = reinterpret_cast<double*>(take(sizeof(double) * L));
    D.part = reinterpret_cast<double*>(take(sizeof(double) * 3 * (size_t)D.cg_blocks));
    D.scal = reinterpret_cast<double*>(take(sizeof(double) * 16));
    if (off > kScratchBytes)
        return fail(c, SMM_EINVAL, "smm_apply_G_noalloc: the problem needs " + std::to_string(off) +
                                       " bytes of work memory, more than the " + std::to_string(kScratchBytes) +
                                       " the no-allocation entry point holds");
    HIPCHK(c, hipMemcpyAsync(D.varphi, varphi_in, sizeof(double) * L, hipMemcpyDeviceToDevice, c->stream));
    int its = 0;
    int rc = eval_G(prob, precision == SMM_FP64, false, true, 0, inner_tol, max_inner, &its);
    if (rc) return rc;
    HIPCHK(c, hipMemcpyAsync(varphi_out, D.x, sizeof(double) * L, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SMM_OK;
}

int smm_debug_cg_system(smm_problem* prob, int* nc, int* nnz, int* rowptr, int* col, double* val, int* map) {
    if (!prob || !nc || !nnz) return SMM_EINVAL;
    if (prob->P.general) return fail(prob->P.ctx, SMM_EUNSUPPORTED, "the CG moment system needs a structured mesh");
    int rc = ensure_host(prob);
    if (rc) return rc;
    Problem& P = prob->P;
    if (!P.cg_ready) {
        assemble_cg(P);
        prob->D.cg_dirty = true;
    }
    *nc = P.cg_nc;
    *nnz = (int)P.cg_col.size();
    if (rowptr) {
        if (!col || !val || !map) return fail(P.ctx, SMM_EINVAL, "smm_debug_cg_system: col, val and map needed");
        std::memcpy(rowptr, P.cg_rowptr.data(), sizeof(int) * P.cg_rowptr.size());
        std::memcpy(col, P.cg_col.data(), sizeof(int) * P.cg_col.size());
        std::memcpy(val, P.cg_val.data(), sizeof(double) * P.cg_val.size());
        std::memcpy(map, P.cg_map.data(), sizeof(int) * P.cg_map.size());
    }
    return SMM_OK;
}

int smm_debug_cg_mg_level(smm_problem* prob, int level, double* A9, int* nvx, int* nvy) {
    if (!prob || level < 0 || !nvx || !nvy) return SMM_EINVAL;
    if (prob->P.general) return fail(prob->P.ctx, SMM_EUNSUPPORTED, "the CG moment system needs a structured mesh");
    int rc = ensure_host(prob);
    if (rc) return rc;
    MGHost M;
    std::string err;
    if ((rc = build_mg_cg(prob->P, M, err))) return fail(prob->P.ctx, rc, err);
    if (level >= (int)M.lev.size()) return fail(prob->P.ctx, SMM_EINVAL, "level beyond the coarsest");
    const MGLevelHost& L = M.lev[level];
    *nvx = L.nvx;
    *nvy = L.nvy;
    if (A9) std::copy(L.A.begin(), L.A.end(), A9);
    return SMM_OK;
}

int smm_debug_cg_spmv(smm_problem* prob, const double* x, double* y) {
    if (!prob || !x || !y) return SMM_EINVAL;
    int rc = ensure_device(prob, true, per_element_forced(prob->D));
    if (rc) return rc;
    if ((rc = ensure_cg(prob))) return rc;
    smm_ctx* c = prob->P.ctx;
    Dev& D = prob->D;
    const CgsArgs a = cgs_args(prob);
    const size_t bytes = sizeof(double) * (size_t)a.nc;
    HIPCHK(c, hipMemcpyAsync(D.cg_p, x, bytes, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, cgs_spmv(a, D.cg_p, D.cg_q, c->stream));
    HIPCHK(c, hipMemcpyAsync(y, D.cg_q, bytes, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SMM_OK;
}

int smm_time_cg_spmv(smm_problem* prob, int reps, double* ms_avg) {
    if (!prob || !ms_avg || reps < 1) return SMM_EINVAL;
    int rc = ensure_device(prob, true, per_element_forced(prob->D));
    if (rc) return rc;
    if ((rc = ensure_cg(prob))) return rc;
    smm_ctx* c = prob->P.ctx;
    Dev& D = prob->D;
    const CgsArgs a = cgs_args(prob);
    std::vector<double> ones((size_t)a.nc, 1.0);
    HIPCHK(c, hipMemcpyAsync(D.cg_p, ones.data(), sizeof(double) * ones.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, cgs_spmv(a, D.cg_p, D.cg_q, c->stream));  // warm-up
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    HIPCHK(c, hipEventRecord(e0, c->stream));
    for (int k = 0; k < reps; ++k) HIPCHK(c, cgs_spmv(a, D.cg_p, D.cg_q, c->stream));
    HIPCHK(c, hipEventRecord(e1, c->stream));
    HIPCHK(c, hipEventSynchronize(e1));
    float ms = 0.0f;
    HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms_avg = ms / reps;
    return SMM_OK;
}

int smm_debug_ip_dense(const smm_problem* prob_c, double* A, double* b_fixed) {
    smm_problem* prob = const_cast<smm_problem*>(prob_c);
    if (!prob) return SMM_EINVAL;
    int rc = ensure_host(prob);
    if (rc) return rc;
    Problem& P = prob->P;
    const long N = (long)P.ne * P.n;
    if (N > 20000) return fail(P.ctx, SMM_EINVAL, "problem too large for a dense copy");
    if (A) {
        std::memset(A, 0, sizeof(double) * N * N);
        for (int K = 0; K < P.ne; ++K)
            for (int s = 0; s < 5; ++s) {
                const int Kc = P.bsr_col[K * 5 + s];
                if (Kc < 0) continue;
                for (int i = 0; i < P.n; ++i)
                    for (int j = 0; j < P.n; ++j)
                        A[((long)K * P.n + i) * N + (long)Kc * P.n + j] +=
                            P.bsr_val[(((size_t)K * 5 + s) * P.n + i) * P.n + j];
            }
    }
    if (b_fixed) std::memcpy(b_fixed, P.b_fixed.data(), sizeof(double) * N);
    return SMM_OK;
}

int smm_debug_sweep_graph(smm_problem* prob, int* level, unsigned char* upstream) {
    if (!prob) return SMM_EINVAL;
    Problem& P = prob->P;
    std::string err;
    int rc = ensure_heavy(P, &err);
    if (rc) return fail(P.ctx, rc, err.empty() ? std::string("geometry setup failed") : err);
    const int nl = P.nlev_max, nt = P.ntiles;
    for (int d = 0; d < P.nd; ++d) {
        if (level)
            for (int t = 0; t < nt; ++t) {
                const int* lp = &P.lev_ptr[((size_t)d * nt + t) * (nl + 1)];
                for (int l = 0; l < nl; ++l)
                    for (int e = lp[l]; e < lp[l + 1]; ++e) level[(size_t)d * P.ne + P.lev_elem[(size_t)d * P.ne + e]] = l;
            }
        if (upstream)
            for (int K = 0; K < P.ne; ++K) upstream[(size_t)d * P.ne + K] = P.upflag[(size_t)d * P.ne + K];
    }
    return SMM_OK;
}

int smm_debug_typed_dense(smm_problem* prob, double* A, double* C, double* b_fixed) {
    if (!prob) return SMM_EINVAL;
    int rc = ensure_typed(prob);
    if (rc) return rc;
    Problem& P = prob->P;
    const long n = P.n, N = (long)P.ne * n;
    if (N > 20000) return fail(P.ctx, SMM_EINVAL, "problem too large for a dense copy");
    auto nbr_of = [&](int K, int f) { return f == 0 ? K - P.nx : f == 1 ? K + 1 : f == 2 ? K + P.nx : K - 1; };
    if (A) std::memset(A, 0, sizeof(double) * N * N);
    if (C) std::memset(C, 0, sizeof(double) * N * 3 * N);
    for (int K = 0; K < P.ne; ++K)
        for (int s = 0; s < 5; ++s) {
            int Kc, t;
            if (s == 0) { Kc = K; t = P.sid[K]; }
            else { t = P.nid[(size_t)K * 4 + s - 1]; if (t < 0) continue; Kc = nbr_of(K, s - 1); }
            const double* ab = (s == 0 ? P.t_ip_self.data() : P.t_ip_nbr.data()) + (size_t)t * n * n;
            const double* cb = (s == 0 ? P.t_c_self.data() : P.t_c_nbr.data()) + (size_t)t * n * 3 * n;
            for (int i = 0; i < n; ++i) {
                if (A)
                    for (int j = 0; j < n; ++j) A[((long)K * n + i) * N + (long)Kc * n + j] += ab[i * n + j];
                if (C)
                    for (int cc = 0; cc < 3; ++cc)
                        for (int j = 0; j < n; ++j)
                            C[((long)K * n + i) * 3 * N + cc * N + (long)Kc * n + j] += cb[i * 3 * n + cc * n + j];
            }
        }
    if (b_fixed) std::memcpy(b_fixed, P.t_bfix.data(), sizeof(double) * N);
    return SMM_OK;
}

int smm_debug_corr_dense(smm_problem* prob, double* C) {
    if (!prob || !C) return SMM_EINVAL;
    int rc = ensure_host(prob);
    if (rc) return rc;
    Problem& P = prob->P;
    const long n = P.n, N = (long)P.ne * n;
    if (N > 20000) return fail(P.ctx, SMM_EINVAL, "problem too large for a dense copy");
    std::memset(C, 0, sizeof(double) * N * 3 * N);
    for (int K = 0; K < P.ne; ++K)
        for (int s = 0; s < 5; ++s) {
            const int Kc = P.bsr_col[K * 5 + s];
            if (Kc < 0) continue;
            const double* cb = &P.corr_val[((size_t)K * 5 + s) * n * 3 * n];
            for (int i = 0; i < n; ++i)
                for (int cc = 0; cc < 3; ++cc)
                    for (int j = 0; j < n; ++j)
                        C[((long)K * n + i) * 3 * N + cc * N + (long)Kc * n + j] += cb[i * 3 * n + cc * n + j];
        }
    return SMM_OK;
}

int smm_time_sweep_parts(smm_problem* prob, int precision, int reps, double* ms_setup, double* ms_particular,
                         double* ms_levels) {
    if (!prob || !ms_setup || !ms_particular || !ms_levels || reps < 1) return SMM_EINVAL;
    int rc = ensure_device(prob, false, per_element_forced(prob->D));
    if (rc) return rc;
    Problem& P = prob->P;
    Dev& D = prob->D;
    smm_ctx* c = P.ctx;
    if (P.cartesian && !per_element_forced(D) && P.tile_x == 0)
        return fail(c, SMM_EUNSUPPORTED, "smm_time_sweep_parts: this problem sweeps with the tabulated kernel");
    if (D.force_general > 1)
        return fail(c, SMM_EUNSUPPORTED, "smm_time_sweep_parts: the sweep path assembles per element");
    const bool fp64 = precision == SMM_FP64;
    bool use = false;
    if ((rc = ensure_inv(prob, fp64, &use))) return rc;
    if (!use) return fail(c, SMM_EUNSUPPORTED, "smm_time_sweep_parts: the stored element operators do not fit");
    const int k = fp64 ? 1 : 0;
    HIPCHK(c, launch_source(fp64, P.ne, P.n, 1, D.sigma_s, D.varphi, nullptr, D.q, D.S, c->stream));
    GenSweepArgs a = gen_args(prob, fp64);
    a.S = D.S;
    a.psibar = P.inflow_layout != SMM_INFLOW_VACUUM ? (fp64 ? D.pbar64 : D.pbar32) : nullptr;
    a.psi = D.psi[0];
    a.invA = D.inv_A[k];
    a.invC = D.inv_C[k];
    a.invG = D.inv_G[k];
    a.inmask = D.inv_mask;
    GenSweepArgs a64 = gen_args(prob, true);
    a64.psibar = P.inflow_layout != SMM_INFLOW_VACUUM ? D.pbar64 : nullptr;
    std::vector<hipEvent_t> ev(6 * reps, nullptr);
    for (hipEvent_t& e : ev) HIPCHK(c, hipEventCreate(&e));
    auto done = [&]() { for (hipEvent_t& e : ev) (void)hipEventDestroy(e); };
    hipError_t e = hipSuccess;
    for (int r = 0; r < reps && e == hipSuccess; ++r) {
        hipEvent_t* t = &ev[6 * r];
        e = hipEventRecord(t[0], c->stream);
        if (e == hipSuccess)
            e = launch_gen_inv_setup(fp64, a64, D.inv_A[k], D.inv_C[k], D.inv_G[k], D.inv_mask, c->stream);
        if (e == hipSuccess) e = hipEventRecord(t[1], c->stream);
        if (e == hipSuccess) e = hipEventRecord(t[2], c->stream);
        if (e == hipSuccess) e = launch_gen_inv_part(fp64, a, 1, c->stream);
        if (e == hipSuccess) e = hipEventRecord(t[3], c->stream);
        if (e == hipSuccess) e = hipEventRecord(t[4], c->stream);
        if (e == hipSuccess) e = launch_gen_inv_part(fp64, a, 2, c->stream);
        if (e == hipSuccess) e = hipEventRecord(t[5], c->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    double sum[3] = {0, 0, 0};
    for (int r = 0; r < reps && e == hipSuccess; ++r)
        for (int q = 0; q < 3 && e == hipSuccess; ++q) {
            float ms = 0;
            e = hipEventElapsedTime(&ms, ev[6 * r + 2 * q], ev[6 * r + 2 * q + 1]);
            sum[q] += ms;
        }
    done();
    if (e != hipSuccess) return fail(c, SMM_EHIP, std::string("smm_time_sweep_parts: ") + hipGetErrorString(e));
    *ms_setup = sum[0] / reps;
    *ms_particular = sum[1] / reps;
    *ms_levels = sum[2] / reps;
    return SMM_OK;
}

int smm_time_sweep(smm_problem* prob, int precision, int reps, double* ms_avg) {
    if (!prob || !ms_avg || reps < 1) return SMM_EINVAL;
    int rc = ensure_device(prob, false, per_element_forced(prob->D));
    if (rc) return rc;
    Problem& P = prob->P;
    Dev& D = prob->D;
    smm_ctx* c = P.ctx;
    const bool fp64 = precision == SMM_FP64;
    const long L = (long)P.ne * P.n;
    HIPCHK(c, launch_source(fp64, P.ne, P.n, 1, D.sigma_s, D.varphi, nullptr, D.q, D.S, c->stream));
    if ((rc = run_sweep(prob, fp64, D.S, 0, nullptr, D.psi[0], true))) return rc;
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    HIPCHK(c, hipEventRecord(e0, c->stream));
    for (int k = 0; k < reps; ++k)
        if ((rc = run_sweep(prob, fp64, D.S, 0, nullptr, D.psi[k & 1], true))) return rc;
    HIPCHK(c, hipEventRecord(e1, c->stream));
    HIPCHK(c, hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)L;
    *ms_avg = ms / reps;
    return SMM_OK;
}

}  // extern "C"
