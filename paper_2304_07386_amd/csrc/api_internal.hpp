// Internal definitions shared by the C-ABI translation units.
#pragma once

#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "smm_internal.hpp"

struct smm_ctx {
    int device = -1;
    hipStream_t stream = nullptr;
    std::string last_error;
};

namespace smm {

// Device-resident state of one problem.
struct Dev {
    bool built = false;
    bool tables_dirty = true;   // materials changed
    bool src_dirty = true;      // source / inflow changed
    std::vector<void*> allocs;
    // quadrature
    double* omega = nullptr;
    void* W32 = nullptr;
    void* W64 = nullptr;
    int ldw = 0;
    // cartesian operator tables
    void *Pm32 = nullptr, *Px32 = nullptr, *Py32 = nullptr;
    void *Pm64 = nullptr, *Px64 = nullptr, *Py64 = nullptr;
    uint8_t* mat = nullptr;
    void *bx32 = nullptr, *by32 = nullptr, *bx64 = nullptr, *by64 = nullptr;
    // general sweep data
    void *Mk32 = nullptr, *Gx32 = nullptr, *Gy32 = nullptr, *nds32 = nullptr, *Lf32 = nullptr, *st32 = nullptr;
    void *Mk64 = nullptr, *Gx64 = nullptr, *Gy64 = nullptr, *nds64 = nullptr, *Lf64 = nullptr, *st64 = nullptr;
    int *nbr = nullptr, *bface_of = nullptr, *lev_ptr = nullptr, *lev_elem = nullptr;
    uint8_t* upflag = nullptr;
    uint8_t* nbr_face = nullptr;          // [ne][4] (meshes given element by element)
    double *w64 = nullptr, *nhat_b = nullptr, *eb0_pt = nullptr;  // boundaries not along x or y
    void *pbar32 = nullptr, *pbar64 = nullptr;
    // materials, source
    double* sigma_s = nullptr;
    double* q = nullptr;
    // moment system
    int* bsr_col = nullptr;
    double *bsr_val = nullptr, *bjac = nullptr, *corr = nullptr, *beta_op = nullptr, *bfix = nullptr;
    int *bface_K = nullptr, *bface_f = nullptr;
    // work vectors
    double *varphi = nullptr, *varphi_prev = nullptr, *x = nullptr, *b = nullptr, *r = nullptr, *z = nullptr,
           *p = nullptr, *qv = nullptr, *part = nullptr, *scal = nullptr, *rpart = nullptr, *rout = nullptr;
    void* S = nullptr;          // sweep source (sized for fp64, [nd_q][ne][n])
    void* psi[2] = {nullptr, nullptr};  // sweep outputs (sized for fp64)
    double *mom = nullptr, *mom_acc = nullptr, *T = nullptr, *beta = nullptr;
    int cg_blocks = 0, r_blocks = 0;
    // continuous (CG) moment system
    int *cg_rowptr = nullptr, *cg_col = nullptr, *cg_tab = nullptr, *cg_map = nullptr;
    double *cg_val = nullptr, *cg_dinv = nullptr, *cg_b = nullptr, *cg_x = nullptr, *cg_r = nullptr,
           *cg_z = nullptr, *cg_p = nullptr, *cg_q = nullptr, *cg_part = nullptr, *cg_scal = nullptr;
    bool cg_dirty = true;   // host CG system rebuilt since the last upload
    hipStream_t cg_cap = nullptr;                 // private stream for graph capture
    std::vector<std::pair<int, hipGraphExec_t>> cg_graphs;  // captured chunks: key 2 k + two-level
    // two-level preconditioner of the CG system (the vertex multigrid levels)
    bool cg_twolevel = false;   // chosen by the solve options
    bool cg_mg_dirty = true;    // CG system rebuilt since the hierarchy was built
    int cg_mg_nlev = 0;
    int cg_mg_nvx[12] = {}, cg_mg_nvy[12] = {};
    double *cg_mg_A[12] = {}, *cg_mg_x[12] = {}, *cg_mg_t[12] = {}, *cg_mg_b[12] = {};
    double* cg_mg_cinv = nullptr;
    double cg_mg_gll[8] = {};
    bool have_outputs = false;
    bool last_typed = false;       // last solve ran on the typed (batched) path
    bool gen_sweep_built = false;  // per-element sweep data uploaded
    bool gen_dirty = true;         // per-element moment system needs (re)upload
    int force_general = 0;
    // stored element operators of the per-element sweep, [0] FP32, [1] FP64
    void* inv_A[2] = {nullptr, nullptr};
    void* inv_C[2] = {nullptr, nullptr};
    void* inv_G[2] = {nullptr, nullptr};
    uint8_t* inv_mask = nullptr;
    bool inv_ready[2] = {false, false};
    bool noalloc_active = false;   // inside smm_apply_G_noalloc: build nothing that needs memory
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};  // phase timing of smm_solve
    double phase_ms[4] = {0, 0, 0, 0};  // source + sweep, moments + closures + rhs, CG, residual
    std::vector<double> hist_r;         // outer residual of each outer iteration of the last smm_solve
    std::vector<int> hist_cg;           // and its CG iterations
    const double* last_mom = nullptr;   // moments of the last G evaluation
    const double* last_varphi = nullptr;
};

}  // namespace smm

struct smm_batch;
struct smm_cnn;

struct smm_problem {
    smm::Problem P;
    smm::Dev D;
    smm_batch* own_batch = nullptr;   // batch of one used by smm_solve on the typed path
    smm_cnn* ws_net = nullptr;        // warm-start network for SMM_START_LEARNED (smm_set_warmstart)
};


namespace smm {
int fail(smm_ctx* c, int code, const std::string& msg);
int batch_solve_single(smm_problem* pr, const smm_solve_opts& o, const double* varphi0, smm_solve_info* info);
// tolerance of the moment solve that builds a diffusion or learned start
double start_tol(const smm_solve_opts& o);
int batch_outputs_single(smm_problem* pr, double* varphi, double* phi, double* J, double* T, double* beta,
                         int on_device);
void batch_release_single(smm_problem* pr);
void batch_history_single(smm_problem* pr, std::vector<double>& r, std::vector<int>& cg);
}  // namespace smm

#define HIPCHK(ctx, call)                                                                        \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return smm::fail(ctx, SMM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)
