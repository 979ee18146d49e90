// Batched SMM solves on uniform Cartesian meshes: many problems of different
// size, order p and S_N set share each kernel launch.
//
//  * the sweep runs as one persistent launch per order p and workgroup size
//    (64-slot chunks of the longest anti-diagonal), whose workgroups take
//    (problem, direction) tasks from a queue ordered by decreasing cost; the
//    launches run one after the other or concurrently on forked streams;
//  * moments, closures, right-hand side, block-Jacobi PCG and the outer
//    residual run as single launches over all problems, with per-problem
//    reductions and convergence flags (problems that have converged drop out
//    of every later launch);
//  * the grid of each persistent sweep launch, and whether the launches
//    share the GPU concurrently, are chosen by timing the candidates on the
//    batch itself (grids cached per launch shape).
// A single problem on the typed path is a batch of one.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <array>
#include <map>
#include <numeric>
#include <tuple>

#include "../../include/smm_cnn.h"
#include "api_internal.hpp"
#include "cnn_internal.hpp"
#include "mg_internal.hpp"

namespace smm {
int ensure_typed(smm_problem* pr);
}

using namespace smm;

namespace {

struct PerProb {
    double *varphi, *varphi_prev, *x, *b, *r, *z, *p, *q, *bfix, *qsrc, *sigma_s, *mom, *mom_acc, *T, *beta;
    int *sid, *nid, *bface_of, *bK, *bF;
    double *ip_self, *ip_nbr, *dinv, *c_self, *c_nbr, *bop, *Lf;
    void* S;
    void* psi;
    double* W64;
    float* W32;
    double* omega;
    double *Pm64, *Px64, *Py64, *bx64, *by64;
    float *Pm32, *Px32, *Py32, *bx32, *by32;
    double* tab64;                   // operator rows in the batched sweep's layout
    float* tab32;
    double *cgw = nullptr, *cgdc = nullptr;  // continuous-space preconditioner term
    uint8_t* mat;
    double* vdiff;
    float* feat0;
    double* gll;
    double *aG, *aF;
};

struct Group {
    int nb = 0, threads = 0;
    bool multi = false;                    // some problem has several materials
    size_t lds[2] = {0, 0};
    int grid[2] = {0, 0};
    // kernel shape per precision: 0 column-wave (b_sweep_kernel), 1 element-lane
    // (b_sweep_elem_kernel, one wave of ethreads / 64 per chunk), 2 and 3 matrix
    // cores (b_sweep_mfma_kernel, FP32 only: 4 and 2 tiles of 16 elements per
    // wave); -1 not tuned
    int shape[2] = {-1, -1};
    int ethreads = 0;
    int maxlen = 0;                        // longest anti-diagonal of the group
    int maxnxy = 0;                        // largest nx + ny of the group
    long maxwords = 0;                     // largest n_elem n_node (one direction's flux)
    std::vector<int2> tasks;
    int2* d_tasks = nullptr;
    int* d_counter = nullptr;
};

// [blocks][rows][cols] row-major -> [blocks][cols][rows]
std::vector<double> col_major(const std::vector<double>& a, int rows, int cols) {
    std::vector<double> t(a.size());
    const size_t bs = (size_t)rows * cols;
    for (size_t b = 0; b < a.size() / bs; ++b)
        for (int i = 0; i < rows; ++i)
            for (int j = 0; j < cols; ++j) t[b * bs + (size_t)j * rows + i] = a[b * bs + (size_t)i * cols + j];
    return t;
}

struct Pool {
    struct Req {
        void** dst;
        size_t off;
    };
    std::vector<Req> reqs;
    size_t total = 0;
    template <typename T>
    void req(T** dst, size_t bytes) {
        reqs.push_back({reinterpret_cast<void**>(dst), total});
        total += (bytes + 255) / 256 * 256;
    }
};

// tuned (grid, kernel shape) per launch shape
std::map<std::tuple<int, int, int, size_t, size_t, int>, std::pair<int, int>>& tune_cache() {
    static std::map<std::tuple<int, int, int, size_t, size_t, int>, std::pair<int, int>> m;
    return m;
}

}  // namespace

struct smm_batch {
    smm_ctx* ctx = nullptr;
    std::vector<smm_problem*> probs;
    int nprob = 0;
    void* pool = nullptr;
    std::vector<PerProb> pp;
    std::vector<BProb> hP;
    BProb* dP = nullptr;
    std::vector<int> blk2p;
    int* d_blk2p = nullptr;
    int nblocks = 0;
    double* part = nullptr;
    std::vector<long> bq0, mw0;
    long* d_bq0 = nullptr;
    long* d_mw0 = nullptr;
    long nbq = 0, nmw = 0;
    int* d_active = nullptr;
    std::vector<int> active;
    double* d_scal = nullptr;
    double* d_rout = nullptr;
    double* d_tol = nullptr;       // per-problem PCG tolerance (inner_adapt)
    // PCG type groups (see BatchLaunch)
    int ngroups = 0;
    int g_nb0[7] = {0, 0, 0, 0, 0, 0, 0};  // group ranges per nb (see BatchLaunch)
    std::vector<int> h_gprob, h_gcount, h_gty, h_gelem;
    int *d_gprob = nullptr, *d_gcount = nullptr, *d_gty = nullptr, *d_gelem = nullptr;
    double* d_gpart = nullptr;
    bool grouped = false;          // groups filled densely enough for the grouped PCG kernels
    bool grouped_auto = false;     // that choice before any testing override
    bool cg_fork = true;           // the per-order PCG launches on forked side streams
    // two-level preconditioner (precond = 1): per-level flat vertex arrays
    bool use_mg = false;
    std::string mg_error;          // why the two-level preconditioner is unavailable (empty: available)
    std::vector<std::vector<double>> gll_host;
    MGLaunch mgl{};
    int* d_mg_off[MG_MAXLEV] = {};
    int* d_mg_dims[MG_MAXLEV] = {};
    double* d_mg_A[MG_MAXLEV] = {};
    double *d_mg_x[MG_MAXLEV] = {}, *d_mg_t[MG_MAXLEV] = {}, *d_mg_b[MG_MAXLEV] = {};
    int *d_mg_lc = nullptr, *d_mg_coff = nullptr;
    int *d_cg_blk2p = nullptr, *d_cg_blk0 = nullptr;  // continuous-space term: node blocks
    double* d_cg_part = nullptr;                      // its per-block partial sums
    std::vector<int> cg_blk2p, cg_blk0, cg_n;         // [blocks], [np], [np] nodes per problem
    double* d_mg_corner = nullptr;
    // Anderson mixing
    double *d_aapart = nullptr, *d_aadot = nullptr, *d_aacoef = nullptr;
    double* d_mg_cinv = nullptr;
    std::vector<Group> groups;
    int* d_sweep_counters = nullptr;  // [groups] task counters of the persistent sweeps
    int sweep_streams[2] = {0, 0};    // per precision: streams the groups run on (0: not tuned yet)
    CartSweepArgs* d_args[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    hipStream_t side[4] = {nullptr, nullptr, nullptr, nullptr};
    hipEvent_t ev_fork = nullptr, ev_join[4] = {nullptr, nullptr, nullptr, nullptr};
    std::vector<smm_solve_info> last_info;
    bool have_outputs = false;
    int ncu = 256;
    // learned warm start
    smm_cnn* ws_net = nullptr;
    bool have_diff = false;
    std::vector<int> ws_used;
    float *d_wsx = nullptr, *d_wsy = nullptr;
    // time of the outer-iteration phases of the last solve (ms): source + sweep,
    // moments + closures + right-hand side, PCG, residual
    hipEvent_t pev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    double phase_ms[4] = {0, 0, 0, 0};
    long cg_batched_its = 0;   // batched PCG iterations launched in the last solve
    bool use_ptol = false;     // PCG stops at the per-problem tolerances d_tol
    std::vector<std::vector<double>> hist;   // per problem: outer residual of each iteration
    std::vector<std::vector<int>> cg_hist;   // per problem: PCG iterations of each outer iteration
    // PCG iteration chunks replayed from captured graphs (use_graph), keyed by
    // (iterations in the chunk, per-problem tolerances on)
    bool use_graph = false;
    hipStream_t cap = nullptr;
    std::map<std::tuple<int, bool, bool, int>, hipGraphExec_t> cg_graphs;  // (chunk, tolerances, two-level, orders)
    // whole outer iterations (use_graph = 2), keyed by (PCG chunk, first sweep,
    // Anderson slot, FP64, per-problem tolerances, two-level, grouped, orders x 8 + sweep streams)
    std::map<std::tuple<int, int, int, int, int, int, int, int>, hipGraphExec_t> it_graphs;
    std::vector<uint8_t> cg_conv;  // per problem: the last PCG reached its tolerance
};

namespace {

BatchLaunch launch_desc(smm_batch* B) {
    BatchLaunch L{};
    L.P = B->dP;
    L.nprob = B->nprob;
    L.blk2p = B->d_blk2p;
    L.nblocks = B->nblocks;
    L.active = B->d_active;
    L.part = B->part;
    L.nbq = B->nbq;
    L.nmw = B->nmw;
    L.bq0 = B->d_bq0;
    L.mw0 = B->d_mw0;
    L.ptol = B->use_ptol ? B->d_tol : nullptr;
    L.ngroups = B->ngroups;
    L.g_prob = B->d_gprob;
    L.g_count = B->d_gcount;
    L.g_ty = B->d_gty;
    L.g_elem = B->d_gelem;
    L.gpart = B->d_gpart;
    for (int k = 0; k < 7; ++k) L.g_nb0[k] = B->g_nb0[k];
    L.order_mask = ~0;
    L.grouped = B->grouped ? 1 : 0;
    L.mg = B->use_mg ? 1 : 0;
    L.mg_corner = B->use_mg ? B->d_mg_corner : nullptr;
    return L;
}

std::vector<float> f32(const std::vector<double>& v) {
    std::vector<float> o(v.size());
    for (size_t i = 0; i < v.size(); ++i) o[i] = (float)v[i];
    return o;
}

// Every device pointer of a descriptor must be set before any kernel reads it.
int check_desc(smm_ctx* c, const BProb& D, int b) {
    const void* ptrs[] = {D.varphi, D.varphi_prev, D.x, D.b, D.r, D.z, D.p, D.q, D.bfix, D.qsrc, D.sigma_s,
                          D.mom, D.mom_acc, D.T, D.beta, D.sid, D.nid, D.bface_of, D.bK, D.bF, D.ip_self,
                          D.ip_nbr, D.dinv, D.c_self, D.c_nbr, D.bop, D.Lf, D.scal, D.S, D.psi, D.W64, D.W32,
                          D.vdiff, D.feat0};
    for (size_t k = 0; k < sizeof(ptrs) / sizeof(ptrs[0]); ++k)
        if (!ptrs[k])
            return fail(c, SMM_EHIP, "batch descriptor " + std::to_string(b) + " field " + std::to_string(k) +
                                         " unset");
    if (D.ldw < D.nd || D.Lpad < D.L || D.Lpad % 4 != 0 || D.nblk < 1) return fail(c, SMM_EHIP, "bad descriptor");
    return SMM_OK;
}

int check_args(smm_ctx* c, const CartSweepArgs& A) {
    if (!A.S || !A.Pm || !A.Px || !A.Py || !A.mat || !A.omega || !A.psi || A.psi_ld < (long)A.nx * A.ny * A.nb * A.nb)
        return fail(c, SMM_EHIP, "bad sweep descriptor");
    return SMM_OK;
}

int put(smm_ctx* c, void* dst, const void* src, size_t bytes) {
    if (!bytes) return SMM_OK;
    if (hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess) return fail(c, SMM_EHIP, "hipMemcpy");
    return SMM_OK;
}

void batch_free(smm_batch* B) {
    if (!B) return;
    if (B->pool) (void)hipFree(B->pool);
    for (void* p : {(void*)B->d_wsx, (void*)B->d_wsy})
        if (p) (void)hipFree(p);
    for (auto& s : B->side)
        if (s) (void)hipStreamDestroy(s);
    if (B->ev_fork) (void)hipEventDestroy(B->ev_fork);
    for (auto& e : B->ev_join)
        if (e) (void)hipEventDestroy(e);
    for (auto& e : B->pev)
        if (e) (void)hipEventDestroy(e);
    for (auto& g : B->cg_graphs) (void)hipGraphExecDestroy(g.second);
    for (auto& g : B->it_graphs) (void)hipGraphExecDestroy(g.second);
    if (B->cap) (void)hipStreamDestroy(B->cap);
    delete B;
}

// psi row stride of a problem: L rounded up to 32 values, so that every row
// starts on a 128-byte line (the moment kernel's 256-byte chunks of a row
// then never share a line with a neighbouring workgroup's chunk: with rows
// aligned to 16 bytes only the line at each chunk boundary was fetched twice)
static size_t psi_row(size_t L) { return (L + 31) / 32 * 32; }

int batch_build(smm_batch* B) {
    smm_ctx* c = B->ctx;
    const int np = B->nprob;
    for (smm_problem* pr : B->probs) {
        int rc = ensure_typed(pr);
        if (rc) return rc;
    }
    (void)hipDeviceGetAttribute(&B->ncu, hipDeviceAttributeMultiprocessorCount, c->device);
    if (B->ncu <= 0) B->ncu = 256;
    B->pp.assign(np, PerProb{});
    B->hP.assign(np, BProb{});
    Pool pool;
    B->bq0.assign(np, 0);
    B->mw0.assign(np, 0);
    B->blk2p.clear();
    long bq = 0, mw = 0;
    for (int b = 0; b < np; ++b) {
        const Problem& P = B->probs[b]->P;
        PerProb& q = B->pp[b];
        const size_t L = (size_t)P.ne * P.n, Lpad = psi_row(L), n = P.n, ne = P.ne;
        const int ldw = (P.nd + 3) / 4 * 4;
        double** v8[] = {&q.varphi, &q.varphi_prev, &q.x, &q.b, &q.r, &q.z, &q.p, &q.q, &q.bfix, &q.qsrc};
        for (double** v : v8) pool.req(v, sizeof(double) * L);
        pool.req(&q.sigma_s, sizeof(double) * ne);
        pool.req(&q.mom, sizeof(double) * 8 * L);
        pool.req(&q.mom_acc, sizeof(double) * 8 * L);
        pool.req(&q.T, sizeof(double) * 3 * L);
        pool.req(&q.beta, sizeof(double) * std::max<size_t>(1, (size_t)P.nbf * P.nq));
        pool.req(&q.sid, sizeof(int) * ne);
        pool.req(&q.nid, sizeof(int) * 4 * ne);
        pool.req(&q.bface_of, sizeof(int) * 4 * ne);
        pool.req(&q.bK, sizeof(int) * std::max(1, P.nbf));
        pool.req(&q.bF, sizeof(int) * std::max(1, P.nbf));
        pool.req(&q.ip_self, sizeof(double) * P.t_ip_self.size());
        pool.req(&q.ip_nbr, sizeof(double) * std::max<size_t>(1, P.t_ip_nbr.size()));
        pool.req(&q.dinv, sizeof(double) * P.t_dinv.size());
        pool.req(&q.c_self, sizeof(double) * P.t_c_self.size());
        pool.req(&q.c_nbr, sizeof(double) * std::max<size_t>(1, P.t_c_nbr.size()));
        pool.req(&q.bop, sizeof(double) * P.t_bop.size());
        pool.req(&q.Lf, sizeof(double) * P.Lf.size());
        pool.req(&q.S, sizeof(double) * L);
        pool.req(&q.psi, sizeof(double) * (size_t)P.nd * Lpad);
        pool.req(&q.W64, sizeof(double) * 16 * ldw);
        pool.req(&q.W32, sizeof(float) * 16 * ldw);
        pool.req(&q.omega, sizeof(double) * P.omega.size());
        pool.req(&q.Pm64, sizeof(double) * P.Pm.size());
        pool.req(&q.Px64, sizeof(double) * P.Px.size());
        pool.req(&q.Py64, sizeof(double) * P.Py.size());
        pool.req(&q.Pm32, sizeof(float) * P.Pm.size());
        pool.req(&q.Px32, sizeof(float) * P.Px.size());
        pool.req(&q.Py32, sizeof(float) * P.Py.size());
        const size_t ntab = (size_t)P.nmat * P.nd * P.n * lane_rw(P.nb);
        pool.req(&q.tab64, sizeof(double) * ntab);
        pool.req(&q.tab32, sizeof(float) * ntab);
        pool.req(&q.bx64, sizeof(double) * (size_t)P.nd * P.ny * P.nb);
        pool.req(&q.by64, sizeof(double) * (size_t)P.nd * P.nx * P.nb);
        pool.req(&q.bx32, sizeof(float) * (size_t)P.nd * P.ny * P.nb);
        pool.req(&q.by32, sizeof(float) * (size_t)P.nd * P.nx * P.nb);
        pool.req(&q.mat, ne);
        pool.req(&q.vdiff, sizeof(double) * L);
        pool.req(&q.aG, sizeof(double) * 3 * L);
        pool.req(&q.aF, sizeof(double) * 3 * L);
        pool.req(&q.feat0, sizeof(float) * 4 * ne);
        // element blocks
        const int epb = 256 / P.n;
        const int nblk = (P.ne + epb - 1) / epb;
        B->hP[b].blk0 = (int)B->blk2p.size();
        B->hP[b].nblk = nblk;
        for (int k = 0; k < nblk; ++k) B->blk2p.push_back(b);
        B->bq0[b] = bq;
        bq += (long)P.nbf * P.nq;
        B->mw0[b] = mw;
        mw += (long)((Lpad + 63) / 64);
    }
    B->nblocks = (int)B->blk2p.size();
    B->nbq = bq;
    B->nmw = mw;
    // PCG type groups: per problem, the elements with one (self, 4 face) type
    // tuple, in chunks of 64 (one wave each)
    B->h_gprob.clear();
    B->h_gcount.clear();
    B->h_gty.clear();
    B->h_gelem.clear();
    // problems in order of nb, so the groups of one order are contiguous
    std::vector<int> by_nb(np);
    for (int b = 0; b < np; ++b) by_nb[b] = b;
    std::stable_sort(by_nb.begin(), by_nb.end(),
                     [&](int a, int b) { return B->probs[a]->P.nb < B->probs[b]->P.nb; });
    for (int k = 0; k < 7; ++k) B->g_nb0[k] = 0;
    for (int b : by_nb) {
        const Problem& P = B->probs[b]->P;
        std::map<std::array<int, 5>, std::vector<int>> tup;
        for (int K = 0; K < P.ne; ++K)
            tup[{P.sid[K], P.nid[4 * K], P.nid[4 * K + 1], P.nid[4 * K + 2], P.nid[4 * K + 3]}].push_back(K);
        B->hP[b].g0 = (int)B->h_gprob.size();
        for (const auto& kv : tup) {
            const std::vector<int>& el = kv.second;
            for (size_t s0 = 0; s0 < el.size(); s0 += 64) {
                const int cnt = (int)std::min<size_t>(64, el.size() - s0);
                B->h_gprob.push_back(b);
                B->h_gcount.push_back(cnt);
                for (int t : kv.first) B->h_gty.push_back(t);
                for (int k = 0; k < 64; ++k) B->h_gelem.push_back(k < cnt ? el[s0 + k] : el[s0]);
            }
        }
        B->hP[b].ng = (int)B->h_gprob.size() - B->hP[b].g0;
        for (int k = P.nb + 1; k < 7; ++k) B->g_nb0[k] = (int)B->h_gprob.size();
    }
    // two-level preconditioner hierarchies (host), flattened per level
    // (a problem it cannot be built for leaves the batch without it: solves
    // that ask for it then fail with the recorded reason)
    std::vector<MGHost> mgh(np);
    B->mg_error.clear();
    for (int b = 0; b < np && B->mg_error.empty(); ++b) {
        std::string err;
        if (build_mg(B->probs[b]->P, mgh[b], err))
            B->mg_error = "two-level preconditioner of problem " + std::to_string(b) + ": " + err;
    }
    int mg_nlev = 0;
    for (const MGHost& m : mgh) mg_nlev = std::max(mg_nlev, (int)m.lev.size());
    if (mg_nlev > MG_MAXLEV) B->mg_error = "mesh too large for the multigrid level table";
    if (!B->mg_error.empty()) {
        mg_nlev = 0;
        for (MGHost& m : mgh) m = MGHost{};
    }
    std::vector<std::vector<int>> mg_off(mg_nlev, std::vector<int>(np + 1, 0)), mg_dims(mg_nlev, std::vector<int>(2 * np, 0));
    std::vector<int> mg_lc(np), mg_coff(np);
    int cinv_tot = 0;
    for (int l = 0; l < mg_nlev; ++l)
        for (int b = 0; b < np; ++b) {
            const bool has = l < (int)mgh[b].lev.size();
            mg_off[l][b + 1] = mg_off[l][b] + (has ? mgh[b].lev[l].nvx * mgh[b].lev[l].nvy : 0);
            mg_dims[l][2 * b] = has ? mgh[b].lev[l].nvx : 0;
            mg_dims[l][2 * b + 1] = has ? mgh[b].lev[l].nvy : 0;
        }
    for (int b = 0; b < np; ++b) {
        mg_lc[b] = std::max((int)mgh[b].lev.size() - 1, 0);
        mg_coff[b] = cinv_tot;
        cinv_tot += (int)mgh[b].cinv.size();
    }
    for (int l = 0; l < mg_nlev; ++l) {
        const size_t nv = (size_t)std::max(mg_off[l][np], 1);
        pool.req(&B->d_mg_off[l], sizeof(int) * (np + 1));
        pool.req(&B->d_mg_dims[l], sizeof(int) * 2 * np);
        pool.req(&B->d_mg_A[l], sizeof(double) * 9 * nv);
        pool.req(&B->d_mg_x[l], sizeof(double) * nv);
        pool.req(&B->d_mg_t[l], sizeof(double) * nv);
        pool.req(&B->d_mg_b[l], sizeof(double) * nv);
    }
    pool.req(&B->d_mg_lc, sizeof(int) * np);
    pool.req(&B->d_aadot, sizeof(double) * 6 * np);
    pool.req(&B->d_aacoef, sizeof(double) * 3 * np);
    {
        long ne_all = 0;
        for (int b = 0; b < np; ++b) {
            B->hP[b].e_off = ne_all;
            ne_all += B->probs[b]->P.ne;
        }
        pool.req(&B->d_mg_corner, sizeof(double) * 4 * std::max(ne_all, 1L));
    }
    pool.req(&B->d_mg_coff, sizeof(int) * np);
    pool.req(&B->d_mg_cinv, sizeof(double) * std::max(cinv_tot, 1));
    // continuous-space term (orders >= 2, with the two-level preconditioner):
    // the continuous Q_p grid of each problem, in blocks of 256 nodes
    B->cg_blk2p.clear();
    B->cg_blk0.assign(np + 1, 0);
    B->cg_n.assign(np, 0);
    for (int b = 0; b < np; ++b) {
        const Problem& P = B->probs[b]->P;
        B->cg_blk0[b] = (int)B->cg_blk2p.size();
        if (!B->mg_error.empty() || P.nb < 3) continue;
        const int p = P.nb - 1;
        B->cg_n[b] = (P.nx * p + 1) * (P.ny * p + 1);
        for (int k = 0; k < (B->cg_n[b] + CG_BLOCK - 1) / CG_BLOCK; ++k) B->cg_blk2p.push_back(b);
        pool.req(&B->pp[b].cgw, sizeof(double) * B->cg_n[b]);
        pool.req(&B->pp[b].cgdc, sizeof(double) * B->cg_n[b]);
    }
    B->cg_blk0[np] = (int)B->cg_blk2p.size();
    pool.req(&B->d_cg_blk2p, sizeof(int) * std::max<size_t>(B->cg_blk2p.size(), 1));
    pool.req(&B->d_cg_blk0, sizeof(int) * (np + 1));
    pool.req(&B->d_cg_part, sizeof(double) * std::max<size_t>(B->cg_blk2p.size(), 1));
    for (int b = 0; b < np; ++b) pool.req(&B->pp[b].gll, sizeof(double) * B->probs[b]->P.nb);
    B->gll_host.assign(np, {});
    for (int b = 0; b < np; ++b) gauss_lobatto01(B->probs[b]->P.p, B->gll_host[b]);
    B->ngroups = (int)B->h_gprob.size();
    {
        // one wave per group pays off when the groups are mostly full (large,
        // piecewise-homogeneous meshes); sparse groups (many material
        // interfaces, small meshes) run the per-node kernels
        long ne_tot = 0;
        for (int b = 0; b < np; ++b) ne_tot += B->probs[b]->P.ne;
        B->grouped = B->ngroups > 0 && (double)ne_tot >= 0.75 * 64.0 * B->ngroups;
        B->grouped_auto = B->grouped;
    }
    pool.req(&B->d_gprob, sizeof(int) * B->ngroups);
    pool.req(&B->d_gcount, sizeof(int) * B->ngroups);
    pool.req(&B->d_gty, sizeof(int) * 5 * B->ngroups);
    pool.req(&B->d_gelem, sizeof(int) * 64 * B->ngroups);
    pool.req(&B->d_gpart, sizeof(double) * 3 * B->ngroups);
    pool.req(&B->dP, sizeof(BProb) * np);
    pool.req(&B->d_blk2p, sizeof(int) * B->nblocks);
    pool.req(&B->part, sizeof(double) * 3 * std::max(B->nblocks, np));
    pool.req(&B->d_aapart, sizeof(double) * 6 * B->nblocks);
    pool.req(&B->d_bq0, sizeof(long) * np);
    pool.req(&B->d_mw0, sizeof(long) * np);
    pool.req(&B->d_active, sizeof(int) * np);
    pool.req(&B->d_scal, sizeof(double) * 16 * np);
    pool.req(&B->d_rout, sizeof(double) * 2 * np);
    pool.req(&B->d_tol, sizeof(double) * np);
    for (int f = 0; f < 2; ++f)
        for (int g = 0; g < 2; ++g) pool.req(&B->d_args[f][g], sizeof(CartSweepArgs) * np);
    // sweep groups by order: the workgroup of a group is NB waves per 64-slot
    // chunk of its longest anti-diagonal (column-wave shape)
    std::map<std::pair<int, int>, int> gi;
    B->groups.clear();
    for (int b = 0; b < np; ++b) {
        const Problem& P = B->probs[b]->P;
        const int th = b_sweep_threads(P.nb, P.nx, P.ny);
        if (th > 1024) return fail(c, SMM_EUNSUPPORTED, "anti-diagonal too long for one workgroup");
        // one group (one persistent launch) per order: its workgroup is sized
        // for the group's longest anti-diagonal, shorter problems leave the
        // extra waves idle.  Problems whose flux exceeds the matrix-core
        // shapes' 32-bit byte offsets form groups of their own, so that a
        // problem takes the same kernel family in any batch
        const int big = (long)P.ne * P.n * (long)sizeof(float) >= (1L << 31) ? 1 : 0;
        const auto key = std::make_pair(P.nb, big);
        if (!gi.count(key)) {
            gi[key] = (int)B->groups.size();
            B->groups.push_back(Group{});
            B->groups.back().nb = P.nb;
        }
        Group& G = B->groups[gi[key]];
        G.threads = std::max(G.threads, th);
        G.ethreads = G.threads / P.nb;   // one wave per chunk
        G.maxlen = std::max(G.maxlen, std::min(P.nx, P.ny));
        G.maxnxy = std::max(G.maxnxy, P.nx + P.ny);
        G.maxwords = std::max(G.maxwords, (long)P.ne * P.n);
        if (P.nmat != 1) G.multi = true;
        for (int d = 0; d < P.nd; ++d) G.tasks.push_back(make_int2(b, d));
    }
    // most work first: with more groups than side streams, the small groups
    // queue behind the large ones instead of the other way round
    {
        auto work = [&](const Group& G) {
            double w = 0;
            for (const int2& t : G.tasks) {
                const Problem& P = B->probs[t.x]->P;
                w += (double)P.ne * P.n;
            }
            return w;
        };
        std::stable_sort(B->groups.begin(), B->groups.end(),
                         [&](const Group& a, const Group& b) { return work(a) > work(b); });
    }
    for (Group& G : B->groups) {
        for (int f = 0; f < 2; ++f) {
            size_t lds = 0;
            for (const int2& t : G.tasks) {
                const Problem& P = B->probs[t.x]->P;
                lds = std::max(lds, b_sweep_lds(f == 1, G.nb, G.multi, P.nx, P.ny));
            }
            G.lds[f] = lds;
        }
        // longest problems first (levels, then anti-diagonal length)
        std::stable_sort(G.tasks.begin(), G.tasks.end(), [&](const int2& a, const int2& b) {
            const Problem& A = B->probs[a.x]->P;
            const Problem& Bp = B->probs[b.x]->P;
            const long ca = (long)(A.nx + A.ny) * 4096 + std::min(A.nx, A.ny);
            const long cb = (long)(Bp.nx + Bp.ny) * 4096 + std::min(Bp.nx, Bp.ny);
            return ca > cb;
        });
        pool.req(&G.d_tasks, sizeof(int2) * G.tasks.size());
    }
    // task counters of all groups in one block (cleared by one launch)
    pool.req(&B->d_sweep_counters, sizeof(int) * std::max<size_t>(B->groups.size(), 1));
    if (hipMalloc(&B->pool, pool.total) != hipSuccess) return fail(c, SMM_ENOMEM, "batch pool allocation");
    for (const auto& r : pool.reqs) *r.dst = static_cast<char*>(B->pool) + r.off;
    for (size_t k = 0; k < B->groups.size(); ++k) B->groups[k].d_counter = B->d_sweep_counters + k;
    if (hipMemset(B->pool, 0, pool.total) != hipSuccess) return fail(c, SMM_EHIP, "hipMemset");
    // uploads and descriptors
    std::vector<CartSweepArgs> args[2][2];
    for (int f = 0; f < 2; ++f)
        for (int g = 0; g < 2; ++g) args[f][g].assign(np, CartSweepArgs{});
    int rc;
    for (int b = 0; b < np; ++b) {
        const Problem& P = B->probs[b]->P;
        PerProb& q = B->pp[b];
        const size_t L = (size_t)P.ne * P.n, Lpad = psi_row(L);
        const int ldw = (P.nd + 3) / 4 * 4;
        std::vector<double> W(16 * (size_t)ldw, 0.0);
        for (int d = 0; d < P.nd; ++d) {
            const double w = P.w[d], ox = P.omega[d * 3], oy = P.omega[d * 3 + 1];
            const double rows[8] = {w, w * ox, w * oy, w * ox * ox, w * ox * oy, w * oy * oy, w * std::fabs(ox),
                                    w * std::fabs(oy)};
            for (int r = 0; r < 8; ++r) W[(size_t)r * ldw + d] = rows[r];
        }
        std::vector<double> bx, by;
        cartesian_boundary_traces(P, bx, by);
        struct U {
            void* d;
            const void* s;
            size_t n;
        };
        // typed blocks go to the device column-major (lanes of one element read
        // consecutive rows of a column)
        const std::vector<double> ip_self_t = col_major(P.t_ip_self, P.n, P.n), ip_nbr_t = col_major(P.t_ip_nbr, P.n, P.n),
                                  dinv_t = col_major(P.t_dinv, P.n, P.n), c_self_t = col_major(P.t_c_self, P.n, 3 * P.n),
                                  c_nbr_t = col_major(P.t_c_nbr, P.n, 3 * P.n), bop_t = col_major(P.t_bop, P.n, P.nq);
        // warm-start features per element: log10 sigma_t, sigma_s / sigma_t,
        // element mean of q, distance of the element centre to the boundary
        std::vector<float> feat0((size_t)4 * P.ne);
        for (int K = 0; K < P.ne; ++K) {
            const int ex = K % P.nx, ey = K / P.nx;
            double qm = 0;
            for (int j = 0; j < P.n; ++j) qm += P.q[(size_t)K * P.n + j];
            const double d = std::min(std::min((ex + 0.5) * P.hx, (P.nx - ex - 0.5) * P.hx),
                                      std::min((ey + 0.5) * P.hy, (P.ny - ey - 0.5) * P.hy));
            feat0[4 * K] = (float)std::log10(P.sigma_t[K]);
            feat0[4 * K + 1] = (float)(P.sigma_s[K] / P.sigma_t[K]);
            feat0[4 * K + 2] = (float)(qm / P.n);
            feat0[4 * K + 3] = (float)d;
        }
        const std::vector<float> W32 = f32(W), Pm32 = f32(P.Pm), Px32 = f32(P.Px), Py32 = f32(P.Py), bx32 = f32(bx),
                                 by32 = f32(by);
        // sweep table: per (material, direction) and node column ca the rows
        // ca + nb b, each [Pm row | Px row | Py row] zero-padded to lane_rw
        const int rw = lane_rw(P.nb);
        std::vector<double> tab((size_t)P.nmat * P.nd * P.n * rw, 0.0);
        for (int o = 0; o < P.nmat * P.nd; ++o)
            for (int ca = 0; ca < P.nb; ++ca)
                for (int bb = 0; bb < P.nb; ++bb) {
                    const int r = ca + P.nb * bb;
                    double* row = &tab[(((size_t)o * P.nb + ca) * P.nb + bb) * rw];
                    for (int cc = 0; cc < P.n; ++cc) row[cc] = P.Pm[((size_t)o * P.n + r) * P.n + cc];
                    for (int cc = 0; cc < P.nb; ++cc) {
                        row[P.n + cc] = P.Px[((size_t)o * P.n + r) * P.nb + cc];
                        row[P.n + P.nb + cc] = P.Py[((size_t)o * P.n + r) * P.nb + cc];
                    }
                }
        const std::vector<float> tab32 = f32(tab);
        const U ups[] = {
            {q.bfix, P.t_bfix.data(), sizeof(double) * L},
            {q.qsrc, P.q.data(), sizeof(double) * L},
            {q.sigma_s, P.sigma_s.data(), sizeof(double) * P.ne},
            {q.sid, P.sid.data(), sizeof(int) * P.ne},
            {q.nid, P.nid.data(), sizeof(int) * 4 * P.ne},
            {q.bface_of, P.bface_of.data(), sizeof(int) * 4 * P.ne},
            {q.bK, P.bface_K.data(), sizeof(int) * P.nbf},
            {q.bF, P.bface_f.data(), sizeof(int) * P.nbf},
            {q.ip_self, ip_self_t.data(), sizeof(double) * ip_self_t.size()},
            {q.ip_nbr, ip_nbr_t.data(), sizeof(double) * ip_nbr_t.size()},
            {q.dinv, dinv_t.data(), sizeof(double) * dinv_t.size()},
            {q.c_self, c_self_t.data(), sizeof(double) * c_self_t.size()},
            {q.c_nbr, c_nbr_t.data(), sizeof(double) * c_nbr_t.size()},
            {q.bop, bop_t.data(), sizeof(double) * bop_t.size()},
            {q.Lf, P.Lf.data(), sizeof(double) * P.Lf.size()},
            {q.W64, W.data(), sizeof(double) * W.size()},
            {q.W32, W32.data(), sizeof(float) * W32.size()},
            {q.omega, P.omega.data(), sizeof(double) * P.omega.size()},
            {q.Pm64, P.Pm.data(), sizeof(double) * P.Pm.size()},
            {q.Px64, P.Px.data(), sizeof(double) * P.Px.size()},
            {q.Py64, P.Py.data(), sizeof(double) * P.Py.size()},
            {q.Pm32, Pm32.data(), sizeof(float) * Pm32.size()},
            {q.Px32, Px32.data(), sizeof(float) * Px32.size()},
            {q.Py32, Py32.data(), sizeof(float) * Py32.size()},
            {q.tab64, tab.data(), sizeof(double) * tab.size()},
            {q.tab32, tab32.data(), sizeof(float) * tab32.size()},
            {q.bx64, bx.data(), sizeof(double) * bx.size()},
            {q.by64, by.data(), sizeof(double) * by.size()},
            {q.bx32, bx32.data(), sizeof(float) * bx32.size()},
            {q.by32, by32.data(), sizeof(float) * by32.size()},
            {q.mat, P.mat_of.data(), P.mat_of.size()},
            {q.feat0, feat0.data(), sizeof(float) * feat0.size()},
        };
        for (const U& u : ups)
            if ((rc = put(c, u.d, u.s, u.n))) return rc;
        BProb& D = B->hP[b];
        D.ne = P.ne; D.n = P.n; D.nb = P.nb; D.nq = P.nq; D.nbf = P.nbf; D.nd = P.nd; D.nx = P.nx; D.ldw = ldw;
        D.L = (long)L; D.Lpad = (long)Lpad; D.eb0x = P.eb0x; D.eb0y = P.eb0y;
        D.bq0 = B->bq0[b]; D.mw0 = B->mw0[b];
        D.varphi = q.varphi; D.varphi_prev = q.varphi_prev; D.x = q.x; D.b = q.b; D.r = q.r; D.z = q.z; D.p = q.p;
        D.q = q.q; D.bfix = q.bfix; D.qsrc = q.qsrc; D.sigma_s = q.sigma_s;
        D.mom = q.mom; D.mom_acc = q.mom_acc; D.T = q.T; D.beta = q.beta;
        D.sid = q.sid; D.nid = q.nid; D.bface_of = q.bface_of; D.bK = q.bK; D.bF = q.bF;
        D.ip_self = q.ip_self; D.ip_nbr = q.ip_nbr; D.dinv = q.dinv; D.c_self = q.c_self; D.c_nbr = q.c_nbr;
        D.bop = q.bop; D.Lf = q.Lf;
        D.scal = B->d_scal + 16 * b;
        D.S = q.S; D.psi = q.psi;
        D.W64 = q.W64; D.W32 = q.W32;
        D.vdiff = q.vdiff; D.feat0 = q.feat0; D.hxhy = P.hx * P.hy;
        D.aG = q.aG; D.aF = q.aF;
        if ((rc = check_desc(c, D, b))) return rc;
        for (int f = 0; f < 2; ++f)
            for (int g = 0; g < 2; ++g) {
                CartSweepArgs& A = args[f][g][b];
                A.nx = P.nx; A.ny = P.ny; A.nd = P.nd; A.nb = P.nb; A.nmat = P.nmat; A.s_aniso = 0;
                A.S = q.S;
                A.Pm = f ? (const void*)q.Pm64 : (const void*)q.Pm32;
                A.Px = f ? (const void*)q.Px64 : (const void*)q.Px32;
                A.Py = f ? (const void*)q.Py64 : (const void*)q.Py32;
                A.tab = f ? (const void*)q.tab64 : (const void*)q.tab32;
                A.mat = q.mat;
                A.omega = q.omega;
                const bool inflow = g == 1 && P.inflow_layout != SMM_INFLOW_VACUUM;
                A.bx = inflow ? (f ? (const void*)q.bx64 : (const void*)q.bx32) : nullptr;
                A.by = inflow ? (f ? (const void*)q.by64 : (const void*)q.by32) : nullptr;
                A.psi = q.psi;
                A.variant = 0;
                A.psi_ld = (long)Lpad;
                if ((rc = check_args(c, A))) return rc;
            }
    }
    for (int g = 0; g < B->ngroups; ++g) {
        const Problem& P = B->probs[B->h_gprob[g]]->P;
        if (B->h_gcount[g] < 1 || B->h_gcount[g] > 64) return fail(c, SMM_EHIP, "bad type group");
        for (int k = 0; k < 64; ++k)
            if (B->h_gelem[64 * (size_t)g + k] < 0 || B->h_gelem[64 * (size_t)g + k] >= P.ne)
                return fail(c, SMM_EHIP, "type group element out of range");
        if (B->h_gty[5 * (size_t)g] < 0 || B->h_gty[5 * (size_t)g] >= P.nself) return fail(c, SMM_EHIP, "bad group type");
        for (int f = 1; f < 5; ++f)
            if (B->h_gty[5 * (size_t)g + f] >= P.nnbrt) return fail(c, SMM_EHIP, "bad group neighbour type");
    }
    if ((rc = put(c, B->d_gprob, B->h_gprob.data(), sizeof(int) * B->ngroups))) return rc;
    if ((rc = put(c, B->d_gcount, B->h_gcount.data(), sizeof(int) * B->ngroups))) return rc;
    if ((rc = put(c, B->d_gty, B->h_gty.data(), sizeof(int) * 5 * B->ngroups))) return rc;
    if ((rc = put(c, B->d_gelem, B->h_gelem.data(), sizeof(int) * 64 * B->ngroups))) return rc;
    // multigrid tables
    for (int l = 0; l < mg_nlev; ++l) {
        if ((rc = put(c, B->d_mg_off[l], mg_off[l].data(), sizeof(int) * (np + 1)))) return rc;
        if ((rc = put(c, B->d_mg_dims[l], mg_dims[l].data(), sizeof(int) * 2 * np))) return rc;
        const int nvl = mg_off[l][np];
        std::vector<double> A((size_t)9 * std::max(nvl, 1), 0.0);
        for (int b = 0; b < np; ++b) {
            if (l >= (int)mgh[b].lev.size()) continue;
            const MGLevelHost& H = mgh[b].lev[l];
            const int nv = H.nvx * H.nvy;
            for (int k = 0; k < 9; ++k)
                for (int v = 0; v < nv; ++v) A[(size_t)k * nvl + mg_off[l][b] + v] = H.A[(size_t)k * nv + v];
        }
        if ((rc = put(c, B->d_mg_A[l], A.data(), sizeof(double) * 9 * nvl))) return rc;
        MGLevelDev& D = B->mgl.lev[l];
        D.off = B->d_mg_off[l];
        D.dims = B->d_mg_dims[l];
        D.A = B->d_mg_A[l];
        D.x = B->d_mg_x[l];
        D.t = B->d_mg_t[l];
        D.b = B->d_mg_b[l];
        D.nv = nvl;
    }
    {
        std::vector<double> cinv;
        for (int b = 0; b < np; ++b) cinv.insert(cinv.end(), mgh[b].cinv.begin(), mgh[b].cinv.end());
        if ((rc = put(c, B->d_mg_lc, mg_lc.data(), sizeof(int) * np))) return rc;
        if ((rc = put(c, B->d_mg_coff, mg_coff.data(), sizeof(int) * np))) return rc;
        if ((rc = put(c, B->d_mg_cinv, cinv.data(), sizeof(double) * cinv.size()))) return rc;
        for (int b = 0; b < np; ++b) {
            if ((rc = put(c, B->pp[b].gll, B->gll_host[b].data(), sizeof(double) * B->gll_host[b].size()))) return rc;
            B->hP[b].gll = B->pp[b].gll;
        }
        B->mgl.nlev = mg_nlev;
        B->mgl.lc = B->d_mg_lc;
        B->mgl.coff = B->d_mg_coff;
        B->mgl.cinv = B->d_mg_cinv;
        B->mgl.omega = 2.0 / 3.0;
        B->mgl.nu = MG_NU;
        // continuous-space term: D_c = diag(P_c^T A P_c) from the typed blocks
        // (row-major on the host): each node's element copies contribute
        // their own diagonal entries, and each face-neighbour pair of copies
        // its coupling entry
        for (int b = 0; b < np; ++b) {
            if (!B->cg_n[b]) continue;
            const Problem& P = B->probs[b]->P;
            const int nb = P.nb, n = P.n, p = nb - 1, nx = P.nx, gx = nx * p + 1;
            std::vector<double> dc((size_t)B->cg_n[b], 0.0);
            auto node = [&](int K, int a) { return ((K / nx) * p + a / nb) * gx + (K % nx) * p + a % nb; };
            const int dK[4] = {-nx, 1, nx, -1};
            for (int K = 0; K < P.ne; ++K) {
                const double* As = &P.t_ip_self[(size_t)P.sid[K] * n * n];
                for (int a = 0; a < n; ++a) dc[node(K, a)] += As[(size_t)a * n + a];
                for (int f = 0; f < 4; ++f) {
                    const int t = P.nid[4 * K + f];
                    if (t < 0) continue;
                    const int N = K + dK[f];
                    const double* An = &P.t_ip_nbr[(size_t)t * n * n];
                    for (int k = 0; k < nb; ++k) {
                        // face node k of K and the node of N at the same place
                        int aK, aN;
                        if (f == 0) { aK = k; aN = k + nb * p; }
                        else if (f == 1) { aK = p + nb * k; aN = nb * k; }
                        else if (f == 2) { aK = k + nb * p; aN = k; }
                        else { aK = nb * k; aN = p + nb * k; }
                        if (node(K, aK) != node(N, aN)) return fail(c, SMM_EHIP, "continuous-space node map");
                        dc[node(K, aK)] += An[(size_t)aK * n + aN];
                    }
                }
            }
            for (double v : dc)
                if (!(v > 0.0)) return fail(c, SMM_EHIP, "continuous-space diagonal not positive");
            if ((rc = put(c, B->pp[b].cgdc, dc.data(), sizeof(double) * dc.size()))) return rc;
        }
        if (!B->cg_blk2p.empty() &&
            (rc = put(c, B->d_cg_blk2p, B->cg_blk2p.data(), sizeof(int) * B->cg_blk2p.size())))
            return rc;
        if ((rc = put(c, B->d_cg_blk0, B->cg_blk0.data(), sizeof(int) * (np + 1)))) return rc;
        B->mgl.cg_blk2p = B->d_cg_blk2p;
        B->mgl.cg_blk0 = B->d_cg_blk0;
        B->mgl.cg_part = B->d_cg_part;
        B->mgl.cg_nblocks = (int)B->cg_blk2p.size();
        for (int b = 0; b < np; ++b) {
            B->hP[b].cgw = B->cg_n[b] ? B->pp[b].cgw : nullptr;
            B->hP[b].cgdc = B->cg_n[b] ? B->pp[b].cgdc : nullptr;
        }
        B->mgl.corner = B->d_mg_corner;
        // first level from which every problem's remaining levels fit in the
        // LDS of one workgroup (three vectors per level)
        B->mgl.ls = mg_nlev;
        B->mgl.lds = 0;
        for (int l = 1; l < mg_nlev; ++l) {
            size_t need = 0;
            for (int b = 0; b < np; ++b) {
                size_t sz = 0;
                for (int k = l; k < (int)mgh[b].lev.size(); ++k)
                    sz += 3 * sizeof(double) * (size_t)mgh[b].lev[k].nvx * mgh[b].lev[k].nvy;
                need = std::max(need, sz);
            }
            if (need <= MG_LDS_CAP) {
                B->mgl.ls = l;
                B->mgl.lds = need;
                break;
            }
        }
        if (B->mgl.ls < mg_nlev && mg_prepare(B->mgl.lds) != hipSuccess)
            return fail(c, SMM_EHIP, "multigrid workgroup LDS size");
        B->mgl.coarse_any = 0;
        for (int b = 0; b < np; ++b)
            if (mg_lc[b] < B->mgl.ls) B->mgl.coarse_any = 1;
    }
    if ((rc = put(c, B->dP, B->hP.data(), sizeof(BProb) * np))) return rc;
    if ((rc = put(c, B->d_blk2p, B->blk2p.data(), sizeof(int) * B->nblocks))) return rc;
    if ((rc = put(c, B->d_bq0, B->bq0.data(), sizeof(long) * np))) return rc;
    if ((rc = put(c, B->d_mw0, B->mw0.data(), sizeof(long) * np))) return rc;
    for (int f = 0; f < 2; ++f)
        for (int g = 0; g < 2; ++g)
            if ((rc = put(c, B->d_args[f][g], args[f][g].data(), sizeof(CartSweepArgs) * np))) return rc;
    for (Group& G : B->groups)
        if ((rc = put(c, G.d_tasks, G.tasks.data(), sizeof(int2) * G.tasks.size()))) return rc;
    B->active.assign(np, 1);
    if ((rc = put(c, B->d_active, B->active.data(), sizeof(int) * np))) return rc;
    for (int k = 0; k < 4; ++k) {
        if (hipStreamCreateWithFlags(&B->side[k], hipStreamNonBlocking) != hipSuccess)
            return fail(c, SMM_EHIP, "hipStreamCreate");
        if (hipEventCreateWithFlags(&B->ev_join[k], hipEventDisableTiming) != hipSuccess)
            return fail(c, SMM_EHIP, "hipEventCreate");
    }
    if (hipEventCreateWithFlags(&B->ev_fork, hipEventDisableTiming) != hipSuccess)
        return fail(c, SMM_EHIP, "hipEventCreate");
    return SMM_OK;
}

// One persistent launch of group G in kernel shape `shape`.
int mfma_threads(const Group& G, int shape) { return b_sweep_mfma_threads(shape == 2 ? 4 : 2, G.maxlen, G.maxlen); }

// the matrix-core shapes address one direction's flux with 32-bit byte offsets
// (buffer descriptors) and take at most four waves
bool mfma_fits(const Group& G, int shape) {
    return mfma_threads(G, shape) <= 256 && G.maxwords * (long)sizeof(float) < (1L << 31);
}

hipError_t group_sweep(smm_batch* B, Group& G, bool fp64, int shape, int grid, const CartSweepArgs* args,
                       hipStream_t s) {
    if (shape >= 2) {
        if (fp64 || !mfma_fits(G, shape)) return hipErrorNotSupported;
        const int tpw = shape == 2 ? 4 : 2, threads = mfma_threads(G, shape);
        return b_sweep_mfma(G.nb, G.multi, tpw, threads, b_sweep_mfma_lds(G.nb, tpw, threads, G.maxnxy), grid,
                            args, G.d_tasks, (int)G.tasks.size(), G.d_counter, B->d_active, s);
    }
    if (shape == 1)
        return b_sweep_elem(fp64, G.nb, G.multi, G.ethreads, grid, args, G.d_tasks, (int)G.tasks.size(), G.d_counter,
                            B->d_active, s);
    return b_sweep(fp64, G.nb, G.multi, G.threads, G.lds[fp64 ? 1 : 0], grid, args, G.d_tasks, (int)G.tasks.size(),
                   G.d_counter, B->d_active, s);
}

// Run the sweep of all active problems: one persistent launch per order, on
// forked streams when there is more than one order.
int batch_sweep(smm_batch* B, bool fp64, bool inflow, hipStream_t st) {
    smm_ctx* c = B->ctx;
    const int f = fp64 ? 1 : 0;
    const int ng = (int)B->groups.size();
    // groups one after the other on the caller's stream, or forked over
    // nstr side streams, or (nstr = 5) the first group (the most work) on the
    // caller's stream, where it is dispatched first, and the others over 3
    // side streams, so that four streams suffice where the process has four
    // hardware queues (chosen by the autotuner)
    const int nstr = std::min(B->sweep_streams[f] > 0 ? B->sweep_streams[f] : 1, 5);
    const bool with_main = nstr == 5;
    const int nside = with_main ? 3 : nstr;
    const bool fork = ng > 1 && nstr > 1;
    const int nfork = std::min(with_main ? ng - 1 : ng, nside);   // side streams in use
    HIPCHK(c, zero_ints(B->d_sweep_counters, ng, st));
    if (fork) {
        HIPCHK(c, hipEventRecord(B->ev_fork, st));
        for (int k = 0; k < nfork; ++k) HIPCHK(c, hipStreamWaitEvent(B->side[k], B->ev_fork, 0));
    }
    for (int k = 0; k < ng; ++k) {
        Group& G = B->groups[k];
        hipStream_t s = !fork ? st : (!with_main ? B->side[k % nside] : (k == 0 ? st : B->side[(k - 1) % nside]));
        int grid = G.grid[f] > 0 ? G.grid[f] : std::min<int>((int)G.tasks.size(), 2 * B->ncu);
        hipError_t e = group_sweep(B, G, fp64, G.shape[f] > 0 ? G.shape[f] : 0, grid, B->d_args[f][inflow ? 1 : 0], s);
        if (e != hipSuccess) return fail(c, SMM_EHIP, std::string("batched sweep: ") + hipGetErrorString(e));
    }
    if (fork)
        for (int k = 0; k < nfork; ++k) {
            HIPCHK(c, hipEventRecord(B->ev_join[k], B->side[k]));
            HIPCHK(c, hipStreamWaitEvent(st, B->ev_join[k], 0));
        }
    return SMM_OK;
}
int batch_sweep(smm_batch* B, bool fp64, bool inflow) { return batch_sweep(B, fp64, inflow, B->ctx->stream); }

// Autotuner: for every persistent sweep launch, time each candidate kernel
// shape (column-wave: NB waves per 64-slot chunk, the node columns of an
// element spread over waves; element-lane: one wave per chunk, each lane a
// whole element; matrix cores: tiles of 16 elements, 4 or 2 tiles per wave,
// FP32 only) and each grid (workgroups per CU), and keep the fastest;
// results are cached per launch shape.  FP32 sweeps choose among the
// matrix-core shapes whenever these fit, so that a problem's result does not
// depend on the batch it is in; within a family, shape and grid only change
// scheduling, not the arithmetic of an element.
int batch_autotune(smm_batch* B, bool fp64) {
    smm_ctx* c = B->ctx;
    const int f = fp64 ? 1 : 0;
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    for (Group& G : B->groups) {
        if (G.grid[f] > 0 && G.shape[f] >= 0) continue;
        auto key = std::make_tuple(G.nb, (int)G.multi + 2 * (G.maxlen + 1024 * (mfma_fits(G, 2) ? 1 : 0)), G.threads,
                                   G.lds[f], G.tasks.size(), f);
        auto it = tune_cache().find(key);
        if (it != tune_cache().end() && G.shape[f] < 0) {
            G.grid[f] = it->second.first;
            G.shape[f] = it->second.second;
            continue;
        }
        int best = 0, best_shape = 0;
        float best_ms = 1e30f;
        const int forced = G.shape[f];   // a shape forced by the testing hook: tune its grid only
        // FP32 sweeps take the matrix-core shapes whenever they fit (their two
        // shapes agree bit for bit, so the choice between them, and the grid,
        // never changes a result); otherwise, and in FP64, the VALU shapes
        const bool mf = !fp64 && (mfma_fits(G, 2) || mfma_fits(G, 3));
        for (int shape = 0; shape < 4; ++shape) {
            if (forced >= 0 && shape != forced) continue;
            if (forced < 0 && mf && shape < 2) continue;
            if (shape == 1 && (G.ethreads < 64 || G.ethreads > 256)) continue;
            if (shape >= 2 && (fp64 || !mfma_fits(G, shape))) continue;
            const std::vector<int> wpcs = shape == 0 ? std::vector<int>{1, 2, 3, 4, 6}
                                                     : std::vector<int>{2, 4, 8, 12, 16};
            for (int wpc : wpcs) {
                const int grid = std::min<int>((int)G.tasks.size(), wpc * B->ncu);
                float ms_tot = 0;
                bool ok = true;
                for (int rep = 0; rep < 3 && ok; ++rep) {
                    HIPCHK(c, zero_ints(G.d_counter, 1, c->stream));
                    HIPCHK(c, hipEventRecord(e0, c->stream));
                    hipError_t e = group_sweep(B, G, fp64, shape, grid, B->d_args[f][1], c->stream);
                    if (e != hipSuccess) {
                        ok = false;
                        (void)hipGetLastError();
                        break;
                    }
                    HIPCHK(c, hipEventRecord(e1, c->stream));
                    HIPCHK(c, hipEventSynchronize(e1));
                    float ms = 0;
                    HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
                    if (rep > 0) ms_tot += ms;
                }
                if (ok && ms_tot < best_ms) {
                    best_ms = ms_tot;
                    best = grid;
                    best_shape = shape;
                }
                if (grid >= (int)G.tasks.size()) break;
            }
        }
        if (best == 0)
            return fail(c, SMM_EUNSUPPORTED, "no launch configuration fits the sweep of order " +
                                                 std::to_string(G.nb - 1) + " (workgroup or LDS limits)");
        G.grid[f] = best;
        G.shape[f] = best_shape;
        if (forced < 0) tune_cache()[key] = std::make_pair(best, best_shape);
    }
    // the groups one after the other, or concurrently on side streams
    if (B->sweep_streams[f] == 0) {
        B->sweep_streams[f] = 1;
        if (B->groups.size() > 1) {
            float best_ms = 1e30f;
            int best = 1;
            for (int ns : {1, 2, 4, 5}) {
                B->sweep_streams[f] = ns;
                float ms_tot = 0;
                for (int rep = 0; rep < 3; ++rep) {
                    HIPCHK(c, hipEventRecord(e0, c->stream));
                    int rc = batch_sweep(B, fp64, true);
                    if (rc) return rc;
                    HIPCHK(c, hipEventRecord(e1, c->stream));
                    HIPCHK(c, hipEventSynchronize(e1));
                    float ms = 0;
                    HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
                    if (rep > 0) ms_tot += ms;
                }
                if (ms_tot < best_ms) {
                    best_ms = ms_tot;
                    best = ns;
                }
            }
            B->sweep_streams[f] = best;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return SMM_OK;
}

// the side streams and events of the PCG iterations' forked per-order
// launches (the sweep's, which are idle while the PCG runs), or none
static const CgFork* cg_fork(smm_batch* B, CgFork& F) {
    if (!B->cg_fork || B->groups.size() < 2) return nullptr;
    for (int k = 0; k < 3; ++k) {
        F.side[k] = B->side[k];
        F.join[k] = B->ev_join[k];
    }
    F.fork = B->ev_fork;
    return &F;
}

// started: the PCG start and done0 iterations were already launched (by an
// outer-iteration graph)
int batch_cg(smm_batch* B, double tol, int max_inner, std::vector<int>& its, bool started = false, int done0 = 0) {
    smm_ctx* c = B->ctx;
    const BatchLaunch L = launch_desc(B);
    if (!started) HIPCHK(c, b_cg_start(L, tol, c->stream, &B->mgl));
    std::vector<double> sc(16 * (size_t)B->nprob);
    // per problem, r.r and the iteration count at the previous check: their
    // ratio gives the residual's reduction per iteration, from which the
    // next chunk is sized so that it ends about when the slowest problem
    // converges (a chunk that overshoots runs iterations with nothing left
    // to do; one that falls short costs one more host round trip)
    std::vector<double> rr_prev(B->nprob, -1.0), it_prev(B->nprob, 0.0);
    int done_its = done0, chunk = 4;
    while (true) {
        HIPCHK(c, hipMemcpyAsync(sc.data(), B->d_scal, sizeof(double) * sc.size(), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        bool all = true;
        int mask = 0;  // orders with problems still iterating
        for (int b = 0; b < B->nprob; ++b) {
            if (!B->active[b]) continue;
            if (sc[16 * b + 6] == 2.0)
                return fail(c, SMM_ENAN, "non-finite values in the moment solve of problem " + std::to_string(b));
            if (sc[16 * b + 6] != 0.0) return fail(c, SMM_EBREAKDOWN, "CG breakdown in problem " + std::to_string(b));
            if (sc[16 * b + 4] == 0.0) {
                all = false;
                mask |= 1 << B->probs[b]->P.nb;
            }
        }
        if (all || done_its >= max_inner) break;
        if (done_its > 0) {
            int need = 1;
            for (int b = 0; b < B->nprob; ++b) {
                const double* q = &sc[16 * (size_t)b];
                if (!B->active[b] || q[4] != 0.0) continue;
                const double rr = q[3], target = q[7], di = q[5] - it_prev[b];
                // no rate known yet: 16 from a fresh start, 2 after the chunk of an
                // iteration graph (which aims just below the iterations needed)
                int nb = started && rr_prev[b] < 0.0 ? 2 : 16;
                if (rr_prev[b] > 0.0 && rr > 0.0 && rr < rr_prev[b] && di > 0.0 && target > 0.0) {
                    const double per = std::log(rr / rr_prev[b]) / di;  // < 0
                    nb = (int)std::ceil(std::log(target / rr) / per);
                }
                need = std::max(need, std::min(std::max(nb, 1), 16));
            }
            // a power of two at most need (few distinct chunk graphs)
            chunk = 1;
            while (chunk * 2 <= need) chunk *= 2;
        }
        for (int b = 0; b < B->nprob; ++b) {
            rr_prev[b] = sc[16 * (size_t)b + 3];
            it_prev[b] = sc[16 * (size_t)b + 5];
        }
        const int k = std::min(chunk, max_inner - done_its);
        // the grouped kernels of orders whose problems have all converged are
        // not launched (they would only check the flags and return)
        BatchLaunch Lk = L;
        Lk.order_mask = mask;
        if (B->use_graph) {
            // capture the chunk once on a private stream, then replay it on the
            // context's stream (kernel nodes only)
            const auto key = std::make_tuple(k, L.ptol != nullptr, L.mg != 0, mask);
            auto it = B->cg_graphs.find(key);
            if (it == B->cg_graphs.end()) {
                if (!B->cap) HIPCHK(c, hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking));
                hipGraph_t g = nullptr;
                hipGraphExec_t ge = nullptr;
                HIPCHK(c, hipStreamBeginCapture(B->cap, hipStreamCaptureModeRelaxed));
                CgFork F;
                const hipError_t e1 = b_cg_iterations(Lk, k, B->cap, &B->mgl, cg_fork(B, F));
                const hipError_t e2 = hipStreamEndCapture(B->cap, &g);
                if (e1 != hipSuccess || e2 != hipSuccess) {
                    if (g) (void)hipGraphDestroy(g);
                    return fail(c, SMM_EHIP, "PCG graph capture failed");
                }
                const hipError_t e3 = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (e3 != hipSuccess) return fail(c, SMM_EHIP, "PCG graph instantiation failed");
                it = B->cg_graphs.emplace(key, ge).first;
            }
            HIPCHK(c, hipGraphLaunch(it->second, c->stream));
        } else {
            CgFork F;
            HIPCHK(c, b_cg_iterations(Lk, k, c->stream, &B->mgl, cg_fork(B, F)));
        }
        done_its += k;
        B->cg_batched_its += k;
    }
    its.assign(B->nprob, 0);
    B->cg_conv.assign(B->nprob, 0);
    for (int b = 0; b < B->nprob; ++b) {
        its[b] = (int)sc[16 * b + 5];
        B->cg_conv[b] = sc[16 * b + 4] != 0.0 ? 1 : 0;
    }
    return SMM_OK;
}

// Warm start: every problem must share nx, ny and the order p.
int ws_dims(smm_batch* B, int* nf, int* nt, int* ny, int* nx) {
    const Problem& P0 = B->probs[0]->P;
    for (const smm_problem* pr : B->probs)
        if (pr->P.nx != P0.nx || pr->P.ny != P0.ny || pr->P.n != P0.n)
            return fail(B->ctx, SMM_EUNSUPPORTED, "warm start needs one mesh size and order for the whole batch");
    *nf = 5 + P0.n;
    *nt = 2 * P0.n;
    *ny = P0.ny;
    *nx = P0.nx;
    return SMM_OK;
}

// varphi_D: the moment system with zero correction source, kept per problem.
int batch_diffusion(smm_batch* B, double tol, int max_inner, std::vector<int>& its) {
    smm_ctx* c = B->ctx;
    HIPCHK(c, b_start_vectors(launch_desc(B), 4, c->stream));   // b = bfix, x = 0
    int rc;
    if ((rc = batch_cg(B, tol, max_inner, its))) return rc;
    HIPCHK(c, b_ws_store_diffusion(launch_desc(B), c->stream));
    B->have_diff = true;
    return SMM_OK;
}

// Learned start: the network predicts, from the features of the diffusion
// start, the nodal correction of the converged flux over it; the start is
// varphi_D + s_K * prediction.  A problem whose prediction is not finite keeps
// the diffusion start.  Adds the CG iterations spent on varphi_D.
int learned_start(smm_batch* B, const smm_solve_opts& o, std::vector<int>& cg_its) {
    smm_ctx* c = B->ctx;
    smm_cnn* net = B->ws_net;
    const int np = B->nprob;
    if (!net) return fail(c, SMM_ESTATE, "SMM_START_LEARNED without smm_batch_set_warmstart");
    int nf, nt, ny, nx, rc;
    if ((rc = ws_dims(B, &nf, &nt, &ny, &nx))) return rc;
    if (net->ctx != c || net->ch[0] != nf || net->ch[net->L] != nt || net->H != ny || net->W != nx)
        return fail(c, SMM_EINVAL, "warm-start network does not match the batch");
    const long ne = (long)nx * ny;
    if (!B->d_wsx) {
        if (hipMalloc((void**)&B->d_wsx, sizeof(float) * np * ne * nf) != hipSuccess ||
            hipMalloc((void**)&B->d_wsy, sizeof(float) * np * ne * nt) != hipSuccess)
            return fail(c, SMM_ENOMEM, "warm-start buffers");
    }
    std::vector<int> its;
    if ((rc = batch_diffusion(B, start_tol(o), o.max_inner, its))) return rc;
    for (int b = 0; b < np; ++b) cg_its[b] += its[b];
    const BatchLaunch L = launch_desc(B);
    HIPCHK(c, hipMemsetAsync(B->d_scal, 0, sizeof(double) * 16 * np, c->stream));
    HIPCHK(c, b_ws_features(L, 0, np, B->d_wsx, nf, c->stream));
    for (int first = 0; first < np; first += net->maxB) {
        const int cnt = std::min(net->maxB, np - first);
        if ((rc = cnn_forward_dev(net, B->d_wsx + first * ne * nf, cnt, nullptr, cnt, B->d_wsy + first * ne * nt)))
            return rc;
    }
    HIPCHK(c, b_ws_apply(L, B->d_wsy, nt, c->stream));
    std::vector<double> sc(16 * (size_t)np);
    HIPCHK(c, hipMemcpyAsync(sc.data(), B->d_scal, sizeof(double) * sc.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    B->ws_used.assign(np, 0);
    for (int b = 0; b < np; ++b) B->ws_used[b] = sc[16 * b + 11] == 0.0;
    return SMM_OK;
}

// The outer fixed point for every problem of the batch (eq. fixed-point),
// each problem stopping on its own relative max-norm test.
int batch_solve(smm_batch* B, const smm_solve_opts& o, const double* const* varphi0, smm_solve_info* info) {
    smm_ctx* c = B->ctx;
    const int np = B->nprob;
    const bool fp64 = o.precision == SMM_FP64;
    const bool delta = o.delta_sweeps != 0;
    auto t0 = std::chrono::steady_clock::now();
    int rc;
    if (o.start < SMM_START_ZERO || o.start > SMM_START_LEARNED)
        return fail(c, SMM_EINVAL, "smm_batch_solve: unknown start mode");
    for (const smm_problem* pr : B->probs)
        if (o.kappa_scale != pr->P.kappa_scale)
            return fail(c, SMM_EUNSUPPORTED, "smm_batch_solve: a batch keeps the penalty scale its problems had when "
                                             "it was created");
    if ((rc = batch_autotune(B, fp64))) return rc;
    B->active.assign(np, 1);
    B->ws_used.assign(np, 0);
    if (o.precond != SMM_PRECOND_BJ && o.precond != SMM_PRECOND_TWOLEVEL)
        return fail(c, SMM_EINVAL, "smm_batch_solve: unknown preconditioner");
    if (!(o.start_tol >= 0)) return fail(c, SMM_EINVAL, "smm_batch_solve: start_tol must be >= 0");
    if (o.precond == SMM_PRECOND_TWOLEVEL && !B->mg_error.empty()) return fail(c, SMM_EUNSUPPORTED, B->mg_error);
    B->use_graph = o.use_graph != 0;
    B->use_mg = o.precond == SMM_PRECOND_TWOLEVEL;
    struct GraphReset {
        smm_batch* b;
        ~GraphReset() {
            b->use_graph = false;
            b->use_mg = false;
        }
    } graph_reset{B};
    if ((rc = put(c, B->d_active, B->active.data(), sizeof(int) * np))) return rc;
    const BatchLaunch L = launch_desc(B);
    std::vector<int> its;
    std::vector<smm_solve_info> inf(np, smm_solve_info{});
    // initial guesses (one launch for the batch; given starts copied per problem)
    if (o.start == SMM_START_GIVEN) {
        HIPCHK(c, b_start_vectors(L, 1 | 2, c->stream));
        for (int b = 0; b < np; ++b)
            if (varphi0 && varphi0[b])
                HIPCHK(c, hipMemcpyAsync(B->pp[b].varphi, varphi0[b], sizeof(double) * B->hP[b].L, hipMemcpyDefault,
                                         c->stream));
    } else if (o.start == SMM_START_DIFFUSION) {
        HIPCHK(c, b_start_vectors(L, 1 | 4, c->stream));
    } else {
        HIPCHK(c, b_start_vectors(L, 1 | 2, c->stream));
    }
    std::vector<int> start_its(np, 0);
    if (o.start == SMM_START_DIFFUSION) {
        if ((rc = batch_cg(B, start_tol(o), o.max_inner, its))) return rc;
        HIPCHK(c, b_start_vectors(L, 8, c->stream));   // varphi = x
        for (int b = 0; b < np; ++b) start_its[b] = its[b];
    } else if (o.start == SMM_START_LEARNED) {
        if ((rc = learned_start(B, o, start_its))) return rc;
    }
    for (int b = 0; b < np; ++b) inf[b].cg_iterations_total = start_its[b];
    auto t1 = std::chrono::steady_clock::now();
    std::vector<double> ro(2 * (size_t)np);
    std::vector<double> r_prev(np, 1.0), tol_k(np, o.inner_tol);
    const int aa = std::max(0, std::min(o.anderson, 2));
    std::vector<double> gram(6 * (size_t)np), coef(3 * (size_t)np);
    int nactive = np;
    // per problem: stopped on the outer test with a trusted moment solve
    // (the final status comes from this flag, not from the last residual)
    std::vector<uint8_t> converged(np, 0);
    int it;
    for (auto& e : B->pev)
        if (!e) HIPCHK(c, hipEventCreate(&e));
    for (double& t : B->phase_ms) t = 0;
    B->cg_batched_its = 0;
    B->hist.assign(np, {});
    B->cg_hist.assign(np, {});
    const bool gmode = o.use_graph >= 2;   // the outer iteration from captured graphs
    int kpred = 8;                          // PCG iterations inside the iteration graph
    for (it = 1; it <= o.max_outer && nactive > 0; ++it) {
        const bool first = (it == 1) || !delta;
        const int slot = (it - 1) % 3;
        if (gmode) {
            // One graph per iteration shape: scattering source, sweep (forked
            // per-order launches), moments, closures, right-hand side, PCG
            // start and kpred PCG iterations, residual (and Anderson's store
            // and Gram products), replayed on the context's stream.  The host
            // then checks the moment solves once; any that has not converged
            // gets more PCG chunks, after which the residual is taken again.
            if (o.inner_adapt > 0) {
                for (int b = 0; b < np; ++b) tol_k[b] = std::max(o.inner_tol, o.inner_adapt * r_prev[b]);
                HIPCHK(c, hipMemcpyAsync(B->d_tol, tol_k.data(), sizeof(double) * np, hipMemcpyHostToDevice,
                                         c->stream));
                B->use_ptol = true;
            }
            const BatchLaunch Lg = launch_desc(B);
            int mask = 0;
            for (int b = 0; b < np; ++b)
                if (B->active[b]) mask |= 1 << B->probs[b]->P.nb;
            const int k = std::max(1, std::min(kpred, o.max_inner));
            const int nstr = B->sweep_streams[fp64 ? 1 : 0];
            const auto key = std::make_tuple(k, first ? 1 : 0, aa > 0 ? slot : -1, fp64 ? 1 : 0,
                                             Lg.ptol ? 1 : 0, Lg.mg, Lg.grouped, mask * 8 + nstr);
            auto gi = B->it_graphs.find(key);
            if (gi == B->it_graphs.end()) {
                if (!B->cap) HIPCHK(c, hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking));
                hipGraph_t g = nullptr;
                hipGraphExec_t ge = nullptr;
                hipStream_t cs = B->cap;
                HIPCHK(c, hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
                BatchLaunch Lk = Lg;
                Lk.order_mask = mask;
                CgFork cgf;
                hipError_t e = b_source(fp64, Lg, !first, cs);
                int src = e == hipSuccess ? batch_sweep(B, fp64, first, cs) : SMM_EHIP;
                if (src == SMM_OK) {
                    // (FP32: T formed with the moments)
                    hipError_t ek[8] = {b_moments(fp64, Lg, true, first, cs, !fp64), b_closures_rhs(Lg, cs, !fp64),
                                        b_copy_x(Lg, cs),
                                        b_cg_start(Lg, o.inner_tol, cs, &B->mgl),
                                        b_cg_iterations(Lk, k, cs, &B->mgl, cg_fork(B, cgf)),
                                        b_residual(Lg, B->d_rout, cs),
                                        aa > 0 ? b_aa_store(Lg, slot, cs) : hipSuccess,
                                        aa > 0 ? b_aa_gram(Lg, B->d_aapart, B->d_aadot, cs) : hipSuccess};
                    for (hipError_t x : ek)
                        if (x != hipSuccess) e = x;
                }
                const hipError_t e2 = hipStreamEndCapture(cs, &g);
                if (src != SMM_OK || e != hipSuccess || e2 != hipSuccess) {
                    if (g) (void)hipGraphDestroy(g);
                    B->use_ptol = false;
                    return fail(c, SMM_EHIP, "outer-iteration graph capture failed");
                }
                const hipError_t e3 = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (e3 != hipSuccess) {
                    B->use_ptol = false;
                    return fail(c, SMM_EHIP, "outer-iteration graph instantiation failed");
                }
                gi = B->it_graphs.emplace(key, ge).first;
            }
            HIPCHK(c, hipEventRecord(B->pev[0], c->stream));
            HIPCHK(c, hipGraphLaunch(gi->second, c->stream));
            HIPCHK(c, hipEventRecord(B->pev[1], c->stream));
            B->cg_batched_its += k;
            const long before = B->cg_batched_its;
            rc = batch_cg(B, o.inner_tol, o.max_inner, its, true, k);
            B->use_ptol = false;
            if (rc) return rc;
            HIPCHK(c, hipEventRecord(B->pev[2], c->stream));
            if (B->cg_batched_its != before) {   // more PCG chunks ran: the residual again
                HIPCHK(c, b_residual(L, B->d_rout, c->stream));
                if (aa > 0) {
                    HIPCHK(c, b_aa_store(L, slot, c->stream));
                    HIPCHK(c, b_aa_gram(L, B->d_aapart, B->d_aadot, c->stream));
                }
            }
            HIPCHK(c, hipEventRecord(B->pev[3], c->stream));
            HIPCHK(c, hipMemcpyAsync(ro.data(), B->d_rout, sizeof(double) * ro.size(), hipMemcpyDeviceToHost,
                                     c->stream));
            if (aa > 0)
                HIPCHK(c, hipMemcpyAsync(gram.data(), B->d_aadot, sizeof(double) * gram.size(),
                                         hipMemcpyDeviceToHost, c->stream));
            else
                HIPCHK(c, b_shift(L, c->stream));
            // the next graph's PCG chunk, from the iterations the active moment
            // solves took: iterations launched after every solve has converged
            // cost whole launches, one host check and a short further chunk
            // cost less, so the chunk aims at the slowest solve's count rounded
            // down to an even number (2..64)
            int need = 0;
            for (int b = 0; b < np; ++b)
                if (B->active[b]) need = std::max(need, its[b]);
            kpred = std::max(2, std::min(64, need & ~1));
        } else {
        HIPCHK(c, hipEventRecord(B->pev[0], c->stream));
        HIPCHK(c, b_source(fp64, L, !first, c->stream));
        if ((rc = batch_sweep(B, fp64, first))) return rc;
        HIPCHK(c, hipEventRecord(B->pev[1], c->stream));
        HIPCHK(c, b_moments(fp64, L, true, first, c->stream, !fp64));   // FP32: T formed with the moments
        HIPCHK(c, b_closures_rhs(L, c->stream, !fp64));
        HIPCHK(c, b_copy_x(L, c->stream));
        HIPCHK(c, hipEventRecord(B->pev[2], c->stream));
        if (o.inner_adapt > 0) {
            for (int b = 0; b < np; ++b) tol_k[b] = std::max(o.inner_tol, o.inner_adapt * r_prev[b]);
            HIPCHK(c, hipMemcpyAsync(B->d_tol, tol_k.data(), sizeof(double) * np, hipMemcpyHostToDevice, c->stream));
            B->use_ptol = true;
        }
        rc = batch_cg(B, o.inner_tol, o.max_inner, its);
        B->use_ptol = false;
        if (rc) return rc;
        HIPCHK(c, hipEventRecord(B->pev[3], c->stream));
        HIPCHK(c, b_residual(L, B->d_rout, c->stream));
        HIPCHK(c, hipMemcpyAsync(ro.data(), B->d_rout, sizeof(double) * ro.size(), hipMemcpyDeviceToHost, c->stream));
        if (aa > 0) {
            HIPCHK(c, b_aa_store(L, slot, c->stream));
            HIPCHK(c, b_aa_gram(L, B->d_aapart, B->d_aadot, c->stream));
            HIPCHK(c, hipMemcpyAsync(gram.data(), B->d_aadot, sizeof(double) * gram.size(), hipMemcpyDeviceToHost,
                                     c->stream));
        } else {
            HIPCHK(c, b_shift(L, c->stream));
        }
        }
        HIPCHK(c, hipEventRecord(B->pev[4], c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (aa > 0) {
            // X_{k+1} = sum_i alpha_i G(X_{k-i}), sum alpha_i = 1, minimising
            // |sum alpha_i f_{k-i}|_2 over the last min(k, aa) + 1 iterates
            const int q = std::min(it - 1, aa) + 1;
            for (int b = 0; b < np; ++b) {
                double* cf = &coef[3 * (size_t)b];
                cf[0] = cf[1] = cf[2] = 0.0;
                cf[slot] = 1.0;
                if (!B->active[b] || q < 2) continue;
                const double rb = ro[2 * b + 1] > 0 ? ro[2 * b] / ro[2 * b + 1] : 0.0;
                if (!(rb >= o.outer_tol)) continue;  // converging now: keep G(X_k)
                const double* gm = &gram[6 * (size_t)b];
                auto dot = [&](int i, int j) {
                    if (i > j) std::swap(i, j);
                    static const int idx[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
                    return gm[idx[i][j]];
                };
                int sl[3];
                for (int i = 0; i < q; ++i) sl[i] = ((slot - i) % 3 + 3) % 3;
                double H[9], tr = 0;
                for (int i = 0; i < q; ++i)
                    for (int j = 0; j < q; ++j) H[i * q + j] = dot(sl[i], sl[j]);
                for (int i = 0; i < q; ++i) tr += H[i * q + i];
                for (int i = 0; i < q; ++i) H[i * q + i] += 1e-10 * tr;
                double y[3] = {1, 1, 1};
                // Gaussian elimination (q <= 3), H symmetric positive semidefinite + shift
                bool ok = tr > 0 && std::isfinite(tr);
                for (int col = 0; ok && col < q; ++col) {
                    const double pv = H[col * q + col];
                    if (!(std::fabs(pv) > 0)) {
                        ok = false;
                        break;
                    }
                    for (int r = col + 1; r < q; ++r) {
                        const double f = H[r * q + col] / pv;
                        for (int k2 = col; k2 < q; ++k2) H[r * q + k2] -= f * H[col * q + k2];
                        y[r] -= f * y[col];
                    }
                }
                double al[3] = {0, 0, 0};
                for (int r = q - 1; ok && r >= 0; --r) {
                    double v = y[r];
                    for (int k2 = r + 1; k2 < q; ++k2) v -= H[r * q + k2] * al[k2];
                    al[r] = v / H[r * q + r];
                }
                double ssum = 0, sabs = 0;
                for (int i = 0; i < q; ++i) {
                    ssum += al[i];
                    sabs += std::fabs(al[i]);
                }
                if (!ok || !std::isfinite(ssum) || ssum == 0 || sabs / std::fabs(ssum) > 1e3) continue;
                for (int i = 0; i < q; ++i) cf[sl[i]] = al[i] / ssum;
            }
            if ((rc = put(c, B->d_aacoef, coef.data(), sizeof(double) * coef.size()))) return rc;
            HIPCHK(c, b_aa_mix(L, B->d_aacoef, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));  // before the host updates the active flags
        }
        for (int ph = 0; ph < 4; ++ph) {
            float ms = 0;
            HIPCHK(c, hipEventElapsedTime(&ms, B->pev[ph], B->pev[ph + 1]));
            B->phase_ms[ph] += ms;
        }
        bool changed = false;
        for (int b = 0; b < np; ++b) {
            if (!B->active[b]) continue;
            const double rabs = ro[2 * b], xmax = ro[2 * b + 1];
            const double r = xmax > 0 ? rabs / xmax : (rabs == 0 ? 0.0 : INFINITY);
            inf[b].iterations = it;
            inf[b].residual = r;
            B->hist[b].push_back(r);
            B->cg_hist[b].push_back(its[b]);
            r_prev[b] = std::isfinite(r) ? r : 1.0;
            inf[b].residual_abs = rabs;
            inf[b].cg_iterations_total += its[b];
            inf[b].cg_iterations_max = std::max(inf[b].cg_iterations_max, its[b]);
            // with adaptive inner tolerances a small change can come from a
            // moment solve that stopped early (its start was already within
            // the loose tolerance); convergence counts only from a solve as
            // tight as the one the target residual itself would ask for,
            // else one more iteration runs, with that tolerance
            const double tight = o.inner_adapt > 0 ? std::max(o.inner_tol, o.inner_adapt * o.outer_tol) : o.inner_tol;
            // and only from a moment solve that reached its tolerance (not
            // one stopped by max_inner)
            const bool trusted = (o.inner_adapt <= 0 || tol_k[b] <= tight) && B->cg_conv[b];
            if (!std::isfinite(r) || (r < o.outer_tol && trusted)) {
                converged[b] = std::isfinite(r) ? 1 : 0;
                B->active[b] = 0;
                --nactive;
                changed = true;
            }
        }
        if (changed && nactive > 0)
            if ((rc = put(c, B->d_active, B->active.data(), sizeof(int) * np))) return rc;
    }
    auto t2 = std::chrono::steady_clock::now();
    const double tsolve = std::chrono::duration<double, std::milli>(t2 - t1).count();
    const double tsetup = std::chrono::duration<double, std::milli>(t1 - t0).count();
    int status = SMM_OK;
    for (int b = 0; b < np; ++b) {
        inf[b].t_total_ms = tsolve + tsetup;
        inf[b].t_setup_ms = tsetup;
        inf[b].t_sweep_ms = B->phase_ms[0];
        inf[b].t_moments_ms = B->phase_ms[1];
        inf[b].t_cg_ms = B->phase_ms[2];
        inf[b].t_residual_ms = B->phase_ms[3];
        if (!std::isfinite(inf[b].residual)) status = SMM_ENAN;
        else if (status == SMM_OK && !converged[b]) status = SMM_ENOCONV;
    }
    B->active.assign(np, 1);
    (void)put(c, B->d_active, B->active.data(), sizeof(int) * np);
    B->last_info = inf;
    B->have_outputs = true;
    if (info)
        for (int b = 0; b < np; ++b) info[b] = inf[b];
    if (status == SMM_ENAN) return fail(c, SMM_ENAN, "non-finite residual");
    if (status == SMM_ENOCONV) return fail(c, SMM_ENOCONV, "max_outer reached");
    return SMM_OK;
}

int batch_outputs(smm_batch* B, int b, double* varphi, double* phi, double* J, double* T, double* beta,
                  int on_device) {
    smm_ctx* c = B->ctx;
    if (!B->have_outputs) return fail(c, SMM_ESTATE, "no solve has run");
    const PerProb& q = B->pp[b];
    const BProb& D = B->hP[b];
    const long L = D.L;
    const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (varphi) HIPCHK(c, hipMemcpyAsync(varphi, q.varphi, sizeof(double) * L, k, c->stream));
    if (phi) HIPCHK(c, hipMemcpyAsync(phi, q.mom_acc, sizeof(double) * L, k, c->stream));
    if (J) HIPCHK(c, hipMemcpyAsync(J, q.mom_acc + L, sizeof(double) * 2 * L, k, c->stream));
    if (T) HIPCHK(c, hipMemcpyAsync(T, q.T, sizeof(double) * 3 * L, k, c->stream));
    if (beta && D.nbf > 0) HIPCHK(c, hipMemcpyAsync(beta, q.beta, sizeof(double) * D.nbf * D.nq, k, c->stream));
    if (!on_device) HIPCHK(c, hipStreamSynchronize(c->stream));
    return SMM_OK;
}

}  // namespace

namespace smm {
// Tolerance of the moment solves that build a start (diffusion, learned): a
// start only seeds the fixed point, so with inexact inner solves it is solved
// to the first outer iteration's tolerance, unless the options set another.
double start_tol(const smm_solve_opts& o) {
    if (o.start_tol > 0) return o.start_tol;
    return o.inner_adapt > 0 ? std::max(o.inner_tol, o.inner_adapt) : o.inner_tol;
}


int batch_solve_single(smm_problem* pr, const smm_solve_opts& o, const double* varphi0, smm_solve_info* info) {
    smm_ctx* c = pr->P.ctx;
    if (!pr->own_batch) {
        smm_batch* B = new smm_batch();
        B->ctx = c;
        B->probs = {pr};
        B->nprob = 1;
        int rc = batch_build(B);
        if (rc) {
            batch_free(B);
            return rc;
        }
        pr->own_batch = B;
    }
    double* dv0 = nullptr;
    if (o.start == SMM_START_GIVEN) {
        if (!varphi0) return fail(c, SMM_EINVAL, "varphi0 required");
        dv0 = const_cast<double*>(varphi0);  // host pointer, copied with hipMemcpyDefault
    }
    const double* v0[1] = {dv0};
    pr->own_batch->ws_net = pr->ws_net;
    return batch_solve(pr->own_batch, o, v0, info);
}

void batch_history_single(smm_problem* pr, std::vector<double>& r, std::vector<int>& cg) {
    r.clear();
    cg.clear();
    if (pr->own_batch && !pr->own_batch->hist.empty()) {
        r = pr->own_batch->hist[0];
        cg = pr->own_batch->cg_hist[0];
    }
}

int batch_outputs_single(smm_problem* pr, double* varphi, double* phi, double* J, double* T, double* beta,
                         int on_device) {
    if (!pr->own_batch) return fail(pr->P.ctx, SMM_ESTATE, "no solve has run");
    return batch_outputs(pr->own_batch, 0, varphi, phi, J, T, beta, on_device);
}

void batch_release_single(smm_problem* pr) {
    if (pr && pr->own_batch) {
        batch_free(pr->own_batch);
        pr->own_batch = nullptr;
    }
}

}  // namespace smm

extern "C" {

int smm_batch_create(smm_ctx* ctx, smm_problem* const* probs, int n, smm_batch** out) {
    if (!ctx || !probs || n < 1 || !out) return SMM_EINVAL;
    if (ctx->device < 0) return fail(ctx, SMM_ESTATE, "host-only context");
    smm_batch* B = new smm_batch();
    B->ctx = ctx;
    B->probs.assign(probs, probs + n);
    B->nprob = n;
    for (smm_problem* p : B->probs)
        if (!p || p->P.ctx != ctx) {
            batch_free(B);
            return fail(ctx, SMM_EINVAL, "problems must belong to the batch's context");
        } else if (p->P.tile_x > 0) {
            batch_free(B);
            return fail(ctx, SMM_EUNSUPPORTED, "batches sweep whole meshes: a problem has sweep tiles set");
        }
    int rc = batch_build(B);
    if (rc) {
        batch_free(B);
        return rc;
    }
    *out = B;
    return SMM_OK;
}

int smm_batch_destroy(smm_batch* batch) {
    batch_free(batch);
    return SMM_OK;
}

int smm_batch_solve(smm_batch* batch, const smm_solve_opts* opts, const double* const* varphi0,
                    smm_solve_info* info) {
    if (!batch) return SMM_EINVAL;
    smm_solve_opts o;
    smm_default_opts(&o);
    if (opts) o = *opts;
    if (o.discretization != SMM_DISC_IP)
        return fail(batch->ctx, SMM_EUNSUPPORTED, "smm_batch_solve: batches solve the IP moment system only");
    return batch_solve(batch, o, varphi0, info);
}

int smm_batch_get_outputs(smm_batch* batch, int k, double* varphi, double* phi, double* J, double* T,
                          double* beta, int on_device) {
    if (!batch || k < 0 || k >= batch->nprob) return SMM_EINVAL;
    return batch_outputs(batch, k, varphi, phi, J, T, beta, on_device);
}

int smm_batch_time_sweep(smm_batch* batch, int precision, int reps, double* ms_avg) {
    if (!batch || reps < 1 || !ms_avg) return SMM_EINVAL;
    smm_ctx* c = batch->ctx;
    const bool fp64 = precision == SMM_FP64;
    int rc = batch_autotune(batch, fp64);
    if (rc) return rc;
    const BatchLaunch L = launch_desc(batch);
    HIPCHK(c, b_source(fp64, L, false, c->stream));
    if ((rc = batch_sweep(batch, fp64, true))) return rc;
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    HIPCHK(c, hipEventRecord(e0, c->stream));
    for (int k = 0; k < reps; ++k)
        if ((rc = batch_sweep(batch, fp64, true))) return rc;
    HIPCHK(c, hipEventRecord(e1, c->stream));
    HIPCHK(c, hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms_avg = ms / reps;
    return SMM_OK;
}

int smm_batch_warmstart_dims(const smm_batch* batch, int* n_features, int* n_targets, int* height, int* width) {
    if (!batch) return SMM_EINVAL;
    int nf, nt, ny, nx;
    int rc = ws_dims(const_cast<smm_batch*>(batch), &nf, &nt, &ny, &nx);
    if (rc) return rc;
    if (n_features) *n_features = nf;
    if (n_targets) *n_targets = nt;
    if (height) *height = ny;
    if (width) *width = nx;
    return SMM_OK;
}

int smm_batch_diffusion(smm_batch* batch, double inner_tol, int max_inner) {
    if (!batch || !(inner_tol > 0) || max_inner < 1) return SMM_EINVAL;
    smm_ctx* c = batch->ctx;
    HIPCHK(c, hipSetDevice(c->device));
    batch->active.assign(batch->nprob, 1);
    int rc;
    if ((rc = put(c, batch->d_active, batch->active.data(), sizeof(int) * batch->nprob))) return rc;
    std::vector<int> its;
    if ((rc = batch_diffusion(batch, inner_tol, max_inner, its))) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SMM_OK;
}

int smm_batch_warmstart_features(smm_batch* batch, int first, int count, float* features) {
    if (!batch || !features || first < 0 || count < 1 || first + count > batch->nprob) return SMM_EINVAL;
    smm_ctx* c = batch->ctx;
    int nf, nt, ny, nx, rc;
    if ((rc = ws_dims(batch, &nf, &nt, &ny, &nx))) return rc;
    if (!batch->have_diff) return fail(c, SMM_ESTATE, "smm_batch_warmstart_features needs smm_batch_diffusion");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, b_ws_features(launch_desc(batch), first, count, features, nf, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SMM_OK;
}

int smm_batch_warmstart_targets(smm_batch* batch, int first, int count, float* targets) {
    if (!batch || !targets || first < 0 || count < 1 || first + count > batch->nprob) return SMM_EINVAL;
    smm_ctx* c = batch->ctx;
    int nf, nt, ny, nx, rc;
    if ((rc = ws_dims(batch, &nf, &nt, &ny, &nx))) return rc;
    if (!batch->have_diff || !batch->have_outputs)
        return fail(c, SMM_ESTATE, "smm_batch_warmstart_targets needs smm_batch_diffusion and a solve");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, b_ws_targets(launch_desc(batch), first, count, targets, nt, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SMM_OK;
}

int smm_batch_set_warmstart(smm_batch* batch, smm_cnn* net) {
    if (!batch) return SMM_EINVAL;
    if (net && net->ctx != batch->ctx) return fail(batch->ctx, SMM_EINVAL, "network and batch on different contexts");
    batch->ws_net = net;
    return SMM_OK;
}

int smm_set_warmstart(smm_problem* prob, smm_cnn* net) {
    if (!prob) return SMM_EINVAL;
    if (net && net->ctx != prob->P.ctx) return fail(prob->P.ctx, SMM_EINVAL, "network and problem on different contexts");
    prob->ws_net = net;
    return SMM_OK;
}

int smm_batch_warmstart_used(const smm_batch* batch, int* used) {
    if (!batch || !used) return SMM_EINVAL;
    if (batch->ws_used.size() != (size_t)batch->nprob) return SMM_ESTATE;
    for (int b = 0; b < batch->nprob; ++b) used[b] = batch->ws_used[b];
    return SMM_OK;
}

int smm_batch_history(const smm_batch* batch, int k, int max_len, double* residual, int* cg_iterations, int* len) {
    if (!batch || k < 0 || k >= batch->nprob || max_len < 0 || !len) return SMM_EINVAL;
    if (batch->hist.size() != (size_t)batch->nprob) return SMM_ESTATE;
    const auto& h = batch->hist[k];
    const int n = (int)std::min<size_t>(h.size(), (size_t)max_len);
    for (int i = 0; i < n; ++i) {
        if (residual) residual[i] = h[i];
        if (cg_iterations) cg_iterations[i] = batch->cg_hist[k][i];
    }
    *len = (int)h.size();
    return SMM_OK;
}

int smm_batch_phase_times(const smm_batch* batch, double* ms, long* cg_iterations) {
    if (!batch || !ms) return SMM_EINVAL;
    for (int k = 0; k < 4; ++k) ms[k] = batch->phase_ms[k];
    if (cg_iterations) *cg_iterations = batch->cg_batched_its;
    return SMM_OK;
}

int smm_batch_time_kernel(smm_batch* batch, int kernel, int reps, double* ms_avg) {
    if (!batch || reps < 1 || !ms_avg) return SMM_EINVAL;
    smm_ctx* c = batch->ctx;
    int rc;
    if (kernel == SMM_KERNEL_SWEEP_FP32 || kernel == SMM_KERNEL_SWEEP_FP64)
        return smm_batch_time_sweep(batch, kernel == SMM_KERNEL_SWEEP_FP64 ? SMM_FP64 : SMM_FP32_SWEEP, reps, ms_avg);
    if (kernel != SMM_KERNEL_CG_SPMV && kernel != SMM_KERNEL_MOMENTS_FP32)
        return fail(c, SMM_EINVAL, "smm_batch_time_kernel: unknown kernel");
    if (!batch->have_outputs) return fail(c, SMM_ESTATE, "smm_batch_time_kernel: run smm_batch_solve first");
    HIPCHK(c, hipSetDevice(c->device));
    batch->active.assign(batch->nprob, 1);
    if ((rc = put(c, batch->d_active, batch->active.data(), sizeof(int) * batch->nprob))) return rc;
    const BatchLaunch L = launch_desc(batch);
    if (kernel == SMM_KERNEL_MOMENTS_FP32) {
        // non-accumulating: the work moments only (equal to the accumulated
        // ones when the last solve did not use delta sweeps, and then the
        // same values again)
        hipEvent_t e0, e1;
        HIPCHK(c, hipEventCreate(&e0));
        HIPCHK(c, hipEventCreate(&e1));
        HIPCHK(c, b_moments(false, L, false, false, c->stream));
        HIPCHK(c, hipEventRecord(e0, c->stream));
        for (int k = 0; k < reps; ++k) HIPCHK(c, b_moments(false, L, false, false, c->stream));
        HIPCHK(c, hipEventRecord(e1, c->stream));
        HIPCHK(c, hipEventSynchronize(e1));
        float ms = 0;
        HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        *ms_avg = ms / reps;
        return SMM_OK;
    }
    // a CG state on the last right-hand side (x, b, p untouched by the timed launches
    // except q and the partial sums)
    HIPCHK(c, b_copy_x(L, c->stream));
    HIPCHK(c, b_cg_start(L, 0.0, c->stream, &batch->mgl));
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    HIPCHK(c, b_cg_spmv(L, c->stream));
    HIPCHK(c, hipEventRecord(e0, c->stream));
    for (int k = 0; k < reps; ++k) HIPCHK(c, b_cg_spmv(L, c->stream));
    HIPCHK(c, hipEventRecord(e1, c->stream));
    HIPCHK(c, hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms_avg = ms / reps;
    return SMM_OK;
}

int smm_batch_apply_sweep(smm_batch* batch, int precision, const double* const* S, int k, double* psi_k) {
    if (!batch || !psi_k) return SMM_EINVAL;
    smm_ctx* c = batch->ctx;
    if (precision != SMM_FP64 && precision != SMM_FP32_SWEEP)
        return fail(c, SMM_EINVAL, "smm_batch_apply_sweep: unknown precision");
    if (k < 0 || k >= batch->nprob) return fail(c, SMM_EINVAL, "smm_batch_apply_sweep: problem index out of range");
    const bool fp64 = precision == SMM_FP64;
    HIPCHK(c, hipSetDevice(c->device));
    int rc;
    // the launch configuration of smm_batch_solve: tuned grids and streams
    if ((rc = batch_autotune(batch, fp64))) return rc;
    batch->active.assign(batch->nprob, 1);
    if ((rc = put(c, batch->d_active, batch->active.data(), sizeof(int) * batch->nprob))) return rc;
    for (int b = 0; b < batch->nprob; ++b) {
        const long L = batch->hP[b].L;
        if (fp64) {
            std::vector<double> h(L, 0.0);
            if (S && S[b]) std::copy(S[b], S[b] + L, h.begin());
            if ((rc = put(c, batch->pp[b].S, h.data(), sizeof(double) * L))) return rc;
        } else {
            std::vector<float> h(L, 0.0f);
            if (S && S[b])
                for (long t = 0; t < L; ++t) h[t] = (float)S[b][t];
            if ((rc = put(c, batch->pp[b].S, h.data(), sizeof(float) * L))) return rc;
        }
    }
    if ((rc = batch_sweep(batch, fp64, true))) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const BProb& D = batch->hP[k];
    const size_t cnt = (size_t)D.nd * D.Lpad;
    if (fp64) {
        std::vector<double> h(cnt);
        HIPCHK(c, hipMemcpy(h.data(), batch->pp[k].psi, sizeof(double) * cnt, hipMemcpyDeviceToHost));
        for (int d = 0; d < D.nd; ++d) std::copy(&h[(size_t)d * D.Lpad], &h[(size_t)d * D.Lpad] + D.L, psi_k + (size_t)d * D.L);
    } else {
        std::vector<float> h(cnt);
        HIPCHK(c, hipMemcpy(h.data(), batch->pp[k].psi, sizeof(float) * cnt, hipMemcpyDeviceToHost));
        for (int d = 0; d < D.nd; ++d)
            for (long t = 0; t < D.L; ++t) psi_k[(size_t)d * D.L + t] = h[(size_t)d * D.Lpad + t];
    }
    return SMM_OK;
}

int smm_debug_batch_precond(smm_batch* batch, int precond, const double* const* r, double* const* z) {
    if (!batch || !r || !z) return SMM_EINVAL;
    smm_ctx* c = batch->ctx;
    if (precond == SMM_PRECOND_TWOLEVEL && !batch->mg_error.empty()) return fail(c, SMM_EUNSUPPORTED, batch->mg_error);
    HIPCHK(c, hipSetDevice(c->device));
    batch->active.assign(batch->nprob, 1);
    int rc;
    if ((rc = put(c, batch->d_active, batch->active.data(), sizeof(int) * batch->nprob))) return rc;
    HIPCHK(c, hipMemset(batch->d_scal, 0, sizeof(double) * 16 * batch->nprob));
    for (int b = 0; b < batch->nprob; ++b)
        if ((rc = put(c, batch->pp[b].r, r[b], sizeof(double) * batch->hP[b].L))) return rc;
    batch->use_mg = precond == SMM_PRECOND_TWOLEVEL;
    const BatchLaunch L = launch_desc(batch);
    batch->use_mg = false;
    HIPCHK(c, b_precond(L, &batch->mgl, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int b = 0; b < batch->nprob; ++b)
        HIPCHK(c, hipMemcpy(z[b], batch->pp[b].z, sizeof(double) * batch->hP[b].L, hipMemcpyDeviceToHost));
    batch->have_outputs = false;
    return SMM_OK;
}

int smm_debug_batch_spmv(smm_batch* batch, const double* const* x, double* const* y) {
    if (!batch || !x || !y) return SMM_EINVAL;
    smm_ctx* c = batch->ctx;
    HIPCHK(c, hipSetDevice(c->device));
    batch->active.assign(batch->nprob, 1);
    int rc;
    if ((rc = put(c, batch->d_active, batch->active.data(), sizeof(int) * batch->nprob))) return rc;
    HIPCHK(c, hipMemset(batch->d_scal, 0, sizeof(double) * 16 * batch->nprob));
    for (int b = 0; b < batch->nprob; ++b)
        if ((rc = put(c, batch->pp[b].p, x[b], sizeof(double) * batch->hP[b].L))) return rc;
    const BatchLaunch L = launch_desc(batch);
    HIPCHK(c, b_cg_spmv(L, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int b = 0; b < batch->nprob; ++b)
        HIPCHK(c, hipMemcpy(y[b], batch->pp[b].q, sizeof(double) * batch->hP[b].L, hipMemcpyDeviceToHost));
    batch->have_outputs = false;
    return SMM_OK;
}

int smm_debug_batch_sweep_shape(smm_batch* batch, int shape) {
    if (!batch || shape < -1 || shape > 3) return SMM_EINVAL;
    for (Group& G : batch->groups) {
        if (shape == 1 && (G.ethreads < 64 || G.ethreads > 256))
            return fail(batch->ctx, SMM_EUNSUPPORTED, "element-lane sweep: anti-diagonal longer than 256 slots");
        if (shape >= 2 && !mfma_fits(G, shape))
            return fail(batch->ctx, SMM_EUNSUPPORTED, "matrix-core sweep: anti-diagonal or mesh too large");
        for (int f = 0; f < 2; ++f) {
            // the matrix-core shapes are FP32 only: FP64 sweeps keep the tuned choice
            G.shape[f] = shape >= 2 && f == 1 ? -1 : shape;
            G.grid[f] = 0;
        }
    }
    for (int f = 0; f < 2; ++f) batch->sweep_streams[f] = 0;
    return SMM_OK;
}

int smm_debug_batch_cg_fork(smm_batch* batch, int fork) {
    if (!batch || fork < 0 || fork > 1) return SMM_EINVAL;
    batch->cg_fork = fork == 1;
    for (auto& kv : batch->cg_graphs) (void)hipGraphExecDestroy(kv.second);
    batch->cg_graphs.clear();
    for (auto& kv : batch->it_graphs) (void)hipGraphExecDestroy(kv.second);
    batch->it_graphs.clear();
    return SMM_OK;
}

int smm_debug_batch_grouped(smm_batch* batch, int grouped) {
    if (!batch || grouped < -1 || grouped > 1) return SMM_EINVAL;
    if (grouped == 1 && batch->ngroups == 0) return fail(batch->ctx, SMM_EUNSUPPORTED, "batch has no type groups");
    batch->grouped = grouped < 0 ? batch->grouped_auto : grouped == 1;
    // captured graphs hold the other kernels
    for (auto& kv : batch->cg_graphs) (void)hipGraphExecDestroy(kv.second);
    batch->cg_graphs.clear();
    for (auto& kv : batch->it_graphs) (void)hipGraphExecDestroy(kv.second);
    batch->it_graphs.clear();
    return SMM_OK;
}

int smm_debug_mg_level(smm_problem* prob, int level, double* A9, int* nvx, int* nvy) {
    if (!prob || level < 0 || !nvx || !nvy) return SMM_EINVAL;
    smm_ctx* c = prob->P.ctx;
    int rc = smm::ensure_typed(prob);
    if (rc) return rc;
    MGHost M;
    std::string err;
    if ((rc = build_mg(prob->P, M, err))) return fail(c, rc, err);
    if (level >= (int)M.lev.size()) return fail(c, SMM_EINVAL, "level beyond the coarsest");
    const MGLevelHost& L = M.lev[level];
    *nvx = L.nvx;
    *nvy = L.nvy;
    if (A9) std::copy(L.A.begin(), L.A.end(), A9);
    return SMM_OK;
}

int smm_batch_units(const smm_batch* batch, double* units) {
    if (!batch || !units) return SMM_EINVAL;
    double u = 0;
    for (const smm_problem* p : batch->probs) u += (double)p->P.ne * p->P.nd * p->P.n;
    *units = u;
    return SMM_OK;
}

}  // extern "C"
