// Host driver of the C-ABI library: setup of the operator and of the
// multigrid hierarchies, the multigrid cycle schedule, the block-acoustic
// preconditioner and the flexible GMRES iteration.  Every arithmetic step
// of the solve, the Hessenberg least-squares update included, runs in the
// kernels included below; the host sequences launches and reads a status
// record per Arnoldi step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "ehelm.h"
#include "eh_common.h"
#include "eh_krylov_kernels.h"
#include "eh_mg_kernels.h"
#include "eh_op_kernels.h"
#include "eh_fine3_kernels.h"
#include "eh_stencil3_kernels.h"
#include "eh_transfer3_kernels.h"
#include "eh_setup_kernels.h"
#include "eh_grad_kernels.h"
#include "eh_group_kernels.h"
#include "eh_fused_kernels.h"
#include "eh_coarse_kernels.h"

using namespace eh;

// Per-source partial sums of eh_misfit_noalloc, in a fixed array of the
// library instead of an allocation: each GPU the library runs on holds its
// own copy until the process ends.  Host code reaches a device's copy only
// through the address hipGetSymbolAddress returns with that device current
// (misfit_scratch); the array's name is not a device address on the host.
#define EH_MISFIT_MAX_SOURCES 4096
static __device__ __align__(256) double scratch[EH_MISFIT_MAX_SOURCES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_addr[kMaxDevices] = {};

// Look up the device address of `scratch` on the current device once (at
// context creation); returns false if the runtime refuses.
bool setup_misfit_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return false;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_addr[device]) return true;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return false;
    g_scratch_addr[device] = (double*)ptr;
    return true;
}

double* misfit_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    return g_scratch_addr[device];
}

thread_local std::string g_create_error;

struct HipError {
    hipError_t e;
    const char* where;
};

#define HIPCHK(x)                                                   \
    do {                                                            \
        hipError_t _e = (x);                                        \
        if (_e != hipSuccess) throw HipError{_e, #x};               \
    } while (0)

struct ArgError {
    std::string msg;
};

// A solve met a non-finite value (EH_ERR_STATE; the context stays usable).
struct StateError {
    std::string msg;
};

// One block of the preconditioner on one multigrid level.
struct Level {
    Dims d{};
    Widths w{};              // stencil half widths (levels >= 1)
    bool half = false;       // symmetric stencil: only offsets from the centre on are stored
    void* coef = nullptr;    // levels >= 1: [stored offsets][np] complex, multigrid precision
    void* dinv = nullptr;    // levels >= 1: damping / diagonal, multigrid precision
    void* f = nullptr;       // right-hand side          (nrhs_cap * np)
    void* u = nullptr;       // iterate                  (nrhs_cap * np)
    void* t = nullptr;       // Jacobi ping-pong buffer  (nrhs_cap * np)
    void* r = nullptr;       // residual                 (nrhs_cap * np)
    void* e = nullptr;       // cycle result             (nrhs_cap * np)
    double damp = 0.8;
    int nstored() const { return half ? (w.nst() + 1) / 2 : w.nst(); }
};

// Block-tridiagonal factors of a coarsest level (eh_coarse_kernels.h).
struct BTData {
    BTPart pt{};
    std::vector<int64_t> goff;   // first entry of each group in the group order (nb + 1)
    std::vector<int64_t> offF;   // F_I = [S_I^-1 | -S_I^-1 L_I] in mats
    std::vector<int64_t> offB;   // B_I = -S_I^-1 U_I in mats
    int64_t* offF_d = nullptr;   // offF on the device
    c128* mats = nullptr;
    int* perm = nullptr;         // group order -> point index (N)
    c128* y = nullptr;           // FP64 work vector, nrhs_cap * N
};

struct Block {
    int kind = 0;            // 0..dim-1: A_{kind+1}; dim: H_p
    int nodal_mask = 0;      // bit a: unknowns nodal along axis a
    std::vector<Level> lev;
    void* fw[3] = {nullptr, nullptr, nullptr};   // fine couplings (multigrid precision)
    void* fD = nullptr;                          // fine diagonal (multigrid precision)
    int64_t Nc = 0;
    c128* Ainv = nullptr;                        // coarsest inverse, FP64, row-major (dense solve)
    bool bt = false;                             // coarsest solved block-tridiagonally
    BTData btd;
};

// Largest coarsest grid solved through an explicit dense inverse.
constexpr int64_t kDenseMax = 6000;

dim3 grid_of(const Dims& d) {
    return dim3((unsigned)((d.g[0] + 63) / 64), (unsigned)((d.g[1] + 3) / 4), (unsigned)d.g[2]);
}
const dim3 kBlock(64, 4, 1);

// Workgroup shapes the autotuner chooses from (all 256 threads or fewer,
// the kernels' launch bound); shape 0 is the default.
const int kShapes[][2] = {{64, 4}, {32, 8}, {128, 2}, {256, 1}, {16, 16}, {64, 2}, {32, 4}};
constexpr int kNumShapes = 7;
constexpr int kMaxLevels = 12;

unsigned lin_grid(int64_t n, int threads = 256, int64_t cap = 65535) {
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    return (unsigned)std::min<int64_t>(g, cap);
}

}  // namespace

// Kernel classes for the event timer (eh_timer_enable / eh_timer_read).
enum KernelClass {
    KC_FINE_SWEEP = 0,   // fine-level damped Jacobi sweep (matrix-free)
    KC_FINE_RESID = 1,   // fine-level residual
    KC_COARSE = 2,       // coarse-level stencil sweeps / residuals (Galerkin)
    KC_RESTRICT = 3,
    KC_PROLONG = 4,
    KC_DENSE = 5,        // coarsest dense solve
    KC_OPERATOR = 6,     // y = H x
    KC_DISTRIBUTE = 7,
    KC_COUPLE = 8,
    KC_KRYLOV = 9,       // Gram-Schmidt, scaling, x update
    KC_FINE_FIRST = 10,  // fine-level first sweep from a zero guess
    KC_FINE_DOWN = 11,   // fused down leg on the fine level
    KC_FINE_UP = 12,     // fused up leg on the fine level
    KC_COARSE_DOWN = 13, // fused down legs on coarse levels
    KC_COARSE_UP = 14,   // fused up legs on coarse levels
    KC_COUNT = 15
};

struct eh_ctx {
    int dim = 2;
    int64_t n[3] = {1, 1, 1};
    double h[3] = {1, 1, 1};
    double omega = 1.0;
    eh_opts o{};
    hipStream_t s = nullptr;
    int device = 0;
    Dims dcell{};
    Dims dface[3]{};
    int64_t ncell = 0, ndof = 0, off[4] = {0, 0, 0, 0}, fsize[4] = {0, 0, 0, 0};
    // FP64 coefficients of H, the distributor and the gradient
    double* k1w[3][3] = {};
    c128* k1D[3] = {};
    double* C = nullptr;          // 1/(lambda+mu)
    double* mu = nullptr;         // mu at cells
    c128* mcell = nullptr;        // rho (1 - i gamma/w) at cells
    double* d_vp = nullptr;
    double* d_vs = nullptr;
    double* d_rho = nullptr;
    double* d_gamma = nullptr;
    double* d_lm = nullptr;       // lambda + mu
    Block blk[4];
    int nblocks = 3;
    int nrhs_cap = 0;
    // Krylov workspace
    int kry_nrhs = 0, kry_m = 0;
    c128* V = nullptr;            // (m+1) * nrhs * ndof
    void* Z = nullptr;            // m * nrhs * ndof, multigrid precision
    c128* W = nullptr;            // nrhs * ndof
    c128* partial = nullptr;
    c128* res_partial = nullptr;    // [rhs][workgroups of one operator application]
    c128* dsmall = nullptr;       // small device arrays (coefs, results)
    int kry_nblk = 0;
    // device-side Arnoldi state and the host-visible status records
    // ([m+1][nrhs]: slot j for step j, slot m for a cycle start), one
    // completion event per slot
    ArnState arn{};
    ArnStatus* arn_host = nullptr;    // pinned host memory
    ArnStatus* arn_dev = nullptr;     // the same memory as the device sees it
    std::vector<hipEvent_t> arn_ev;
    void* tmpT = nullptr;         // nrhs * ndof multigrid precision (preconditioner I/O)
    c128* zbuf = nullptr;         // 2 * ndof: work vectors of the Z(alpha) mat-vec
    c128* zy = nullptr;           // ncell: Z v in the power method
    int64_t tmpT_elems = 0;
    double* misfit_part = nullptr; // eh_misfit's per-source partial sums (grown as needed)
    int misfit_cap = 0;
    std::vector<void*> allocs;
    std::string err;
    bool broken = false;
    // event timing of selected kernel classes (eh_timer_enable / eh_timer_read)
    unsigned timer_mask = 0;
    struct TimerRec { int cls; hipEvent_t a, b; double bytes; };
    std::vector<TimerRec> timer_recs;
    std::vector<hipEvent_t> event_pool;
    // captured Arnoldi steps: one graph per step j, valid for graph_nrhs
    // right-hand sides in a solve of graph_stride (the layout stride of the
    // status records and small arrays); used only while no kernel class is
    // being timed
    struct GraphEntry { hipGraphExec_t exec = nullptr; hipGraph_t graph = nullptr; };
    std::vector<GraphEntry> graphs;
    int graph_nrhs = -1;
    int graph_stride = -1;
    bool capturing = false;
    hipStream_t solve_stream = nullptr;
    hipEvent_t order_event = nullptr;      // orders the solve stream after the user's
    // launch shapes per block group (0: H_p, 1: shear blocks), level and
    // kernel kind (0: sweeps/residuals, 1: restriction, 2: prolongation)
    int shape[2][kMaxLevels][3] = {};
    // tile configurations of the fused legs per block group and level
    // (0: down leg, 1: up leg), indices into kFDown / kFUp
    int fcfg[2][kMaxLevels][2] = {};
    int tuned_nrhs = 0;
    bool use_bt = false;          // coarsest levels solved block-tridiagonally (else dense inverse)

    template <class P>
    P* alloc(size_t count) {
        void* p = nullptr;
        if (count == 0) count = 1;
        hipError_t e = hipMalloc(&p, count * sizeof(P));
        if (e != hipSuccess) throw HipError{e, "hipMalloc"};
        allocs.push_back(p);
        return (P*)p;
    }
    void release(void* p) {
        if (!p) return;
        auto it = std::find(allocs.begin(), allocs.end(), p);
        if (it != allocs.end()) allocs.erase(it);
        (void)hipFree(p);
    }
    size_t csize() const { return o.mg_precision == 32 ? sizeof(c64) : sizeof(c128); }
    size_t rsize() const { return o.mg_precision == 32 ? sizeof(float) : sizeof(double); }
};

namespace {

// Events for timing only: without the system-scope fence, recording an event
// does not write back and invalidate the caches around the kernel it brackets.
hipEvent_t take_event(eh_ctx* c) {
    if (!c->event_pool.empty()) {
        hipEvent_t e = c->event_pool.back();
        c->event_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    return e;
}

void drop_graphs(eh_ctx* c) {
    for (auto& g : c->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    c->graphs.clear();
    c->graph_nrhs = -1;
    c->graph_stride = -1;
}

// Records a start event before and a stop event after the launches in its
// scope when the class is selected; `bytes` is the algorithmic traffic.
struct Timed {
    eh_ctx* c;
    int cls;
    double bytes;
    bool on;
    hipEvent_t a{}, b{};
    Timed(eh_ctx* c_, int cls_, double bytes_) : c(c_), cls(cls_), bytes(bytes_) {
        // graphs are only captured with timing off, so events are plain
        on = ((c->timer_mask >> cls) & 1u) && !c->capturing;
        if (on) {
            a = take_event(c);
            b = take_event(c);
            HIPCHK(hipEventRecord(a, c->s));
        }
    }
    ~Timed() {
        if (!on) return;
        if (hipEventRecord(b, c->s) == hipSuccess) c->timer_recs.push_back({cls, a, b, bytes});
        else c->broken = true;     // reported by the next call
    }
};

// ---------------------------------------------------------------------------
// setup on the host (FP64)

struct HostMedium {
    std::vector<double> mu, lm, rho, gamma;
    std::vector<std::complex<double>> m;   // rho (1 - i gamma/w), unshifted
};

int64_t cidx(const eh_ctx* c, int i, int j, int k) {
    return ((int64_t)k * c->n[1] + j) * c->n[0] + i;
}

// gamma = gamma0 + w * sum_a l_a^2, l_a = max(0, W - d_a)/W, d_a the distance
// (cells, centre to side) to the nearest absorbing side along axis a
// (Section 4: a layer of gradually increasing attenuation).
double abc_gamma(const eh_ctx* c, int i, int j, int k) {
    const int idx[3] = {i, j, k};
    double g = c->o.gamma0;
    const int W = c->o.abc_width;
    if (W <= 0) return g;
    for (int a = 0; a < c->dim; ++a) {
        double d = 1e300;
        if (c->o.abc_sides & (1u << (2 * a))) d = std::min(d, idx[a] + 0.5);
        if (c->o.abc_sides & (1u << (2 * a + 1))) d = std::min(d, c->n[a] - idx[a] - 0.5);
        const double l = std::max(0.0, W - d) / W;
        g += c->omega * l * l;
    }
    return g;
}

// Mean of mu over the existing cells around the location whose nodal axes
// are `nodal` (bit mask) at location index (li, lj, lk).
double mu_mean(const eh_ctx* c, const HostMedium& M, int nodal, int li, int lj, int lk) {
    const int L[3] = {li, lj, lk};
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        if (a < c->dim && (nodal & (1 << a))) { lo[a] = L[a] - 1; hi[a] = L[a]; }
        else { lo[a] = L[a]; hi[a] = L[a]; }
    }
    double s = 0.0;
    int cnt = 0;
    for (int z = lo[2]; z <= hi[2]; ++z)
        for (int y = lo[1]; y <= hi[1]; ++y)
            for (int x = lo[0]; x <= hi[0]; ++x) {
                if (x < 0 || y < 0 || z < 0 || x >= c->n[0] || y >= c->n[1] || z >= c->n[2]) continue;
                s += M.mu[cidx(c, x, y, z)];
                ++cnt;
            }
    return s / cnt;
}

// Fine-level acoustic block A_k on the k-faces: couplings w_a (between a
// face and its +e_a neighbour) and the diagonal, from grad_h^T A_e(mu) grad_h
// - w^2 A_f(m) (eq. mixed-discretized); alpha shifts the mass (eq. shift).
void build_Ak(const eh_ctx* c, const HostMedium& M, int kb, double alpha,
              std::vector<double> w[3], std::vector<std::complex<double>>& D) {
    const Dims& d = c->dface[kb];
    const int64_t np = d.np();
    for (int a = 0; a < c->dim; ++a) w[a].assign(np, 0.0);
    D.assign(np, 0.0);
    const double om2 = c->omega * c->omega;
    for (int z = 0; z < d.g[2]; ++z)
        for (int y = 0; y < d.g[1]; ++y)
            for (int x = 0; x < d.g[0]; ++x) {
                const int64_t p = ((int64_t)z * d.g[1] + y) * d.g[0] + x;
                const int P[3] = {x, y, z};
                double stiff = 0.0;
                for (int a = 0; a < c->dim; ++a) {
                    const double ih2 = 1.0 / (c->h[a] * c->h[a]);
                    if (a == kb) {
                        // derivative along the nodal axis lands on cells P[a]-1 and P[a]
                        int q[3] = {x, y, z};
                        if (P[a] < c->n[a]) {
                            const double m = M.mu[cidx(c, q[0], q[1], q[2])] * ih2;
                            w[a][p] = m;
                            stiff += m;
                        }
                        if (P[a] >= 1) {
                            q[a] = P[a] - 1;
                            stiff += M.mu[cidx(c, q[0], q[1], q[2])] * ih2;
                        }
                    } else {
                        // derivative along a cell-centred axis lands on edges at
                        // node indices P[a] and P[a]+1 (zero ghost outside)
                        const int nm = (1 << kb) | (1 << a);
                        int q[3] = {x, y, z};
                        const double m0 = mu_mean(c, M, nm, q[0], q[1], q[2]) * ih2;
                        q[a] = P[a] + 1;
                        const double m1 = mu_mean(c, M, nm, q[0], q[1], q[2]) * ih2;
                        stiff += m0 + m1;
                        if (P[a] + 1 < d.g[a]) w[a][p] = m1;
                    }
                }
                // face mass: mean of the existing cells on both sides along kb
                std::complex<double> mf = 0.0;
                int cnt = 0;
                for (int off = -1; off <= 0; ++off) {
                    int q[3] = {x, y, z};
                    q[kb] += off;
                    if (q[kb] < 0 || q[kb] >= c->n[kb]) continue;
                    const int64_t ci = cidx(c, q[0], q[1], q[2]);
                    mf += M.rho[ci] * std::complex<double>(1.0, -(M.gamma[ci] / c->omega + alpha));
                    ++cnt;
                }
                mf /= double(cnt);
                D[p] = stiff - om2 * mf;
            }
}

// Fine-level H_p on the cells: H_p = B B^T diag(w) - w^2 diag(m/(lambda+mu)),
// w = (lambda + 2 mu)/(lambda + mu) (eqs. Ap, Hp); alpha shifts m.
void build_Hp(const eh_ctx* c, const HostMedium& M, double alpha, std::vector<double>& w,
              std::vector<std::complex<double>>& D) {
    const int64_t nc = c->ncell;
    w.assign(nc, 0.0);
    D.assign(nc, 0.0);
    double sum_ih2 = 0.0;
    for (int a = 0; a < c->dim; ++a) sum_ih2 += 2.0 / (c->h[a] * c->h[a]);
    const double om2 = c->omega * c->omega;
    for (int64_t q = 0; q < nc; ++q) {
        w[q] = 1.0 + M.mu[q] / M.lm[q];
        const std::complex<double> ms = M.rho[q] * std::complex<double>(1.0, -(M.gamma[q] / c->omega + alpha));
        D[q] = w[q] * sum_ih2 - om2 * ms / M.lm[q];
    }
}

template <class T>
void upload_real(eh_ctx* c, void** dst, const std::vector<double>& v) {
    std::vector<T> t(v.begin(), v.end());
    T* p = c->alloc<T>(t.size());
    HIPCHK(hipMemcpy(p, t.data(), t.size() * sizeof(T), hipMemcpyHostToDevice));
    *dst = p;
}

template <class T>
void upload_cplx(eh_ctx* c, void** dst, const std::vector<std::complex<double>>& v) {
    std::vector<cplx<T>> t(v.size());
    for (size_t q = 0; q < v.size(); ++q) t[q] = mk<T>(T(v[q].real()), T(v[q].imag()));
    cplx<T>* p = c->alloc<cplx<T>>(t.size());
    HIPCHK(hipMemcpy(p, t.data(), t.size() * sizeof(cplx<T>), hipMemcpyHostToDevice));
    *dst = p;
}

// FP64 stencil (half widths 1) of a fine block for the Galerkin setup.
// H_p with the Remark's A~_p = B A_f(mu) B^T - w^2 M_p in place of A_p:
// H~_p = B B^T + A~_p C.  Across the face between cell c and its neighbour
// nb along axis a the coupling is (1 + mu_f / (lambda+mu)_nb) / h_a^2, mu_f
// the mean of the face's existing cells (a boundary face has one); the
// diagonal collects (1 + mu_f / (lambda+mu)_c) / h_a^2 over the cell's
// faces and the shifted mass / (lambda+mu)_c.  wpm[a] holds the pair
// (coupling to c + e_a, to c - e_a) per cell.
void build_Hp_tilde(const eh_ctx* c, const HostMedium& M, double alpha, std::vector<double> wpm[3],
                    std::vector<std::complex<double>>& D) {
    const Dims& d = c->dcell;
    const int64_t nc = c->ncell;
    const int64_t st[3] = {1, d.g[0], (int64_t)d.g[0] * d.g[1]};
    for (int a = 0; a < c->dim; ++a) wpm[a].assign(2 * nc, 0.0);
    D.assign(nc, 0.0);
    const double om2 = c->omega * c->omega;
    for (int64_t q = 0; q < nc; ++q) {
        const int P[3] = {(int)(q % d.g[0]), (int)((q / d.g[0]) % d.g[1]), (int)(q / st[2])};
        double diag = 0.0;
        for (int a = 0; a < c->dim; ++a) {
            const double ih2 = 1.0 / (c->h[a] * c->h[a]);
            const bool hi = P[a] + 1 < d.g[a], lo = P[a] > 0;
            const double mhi = hi ? 0.5 * (M.mu[q] + M.mu[q + st[a]]) : M.mu[q];
            const double mlo = lo ? 0.5 * (M.mu[q] + M.mu[q - st[a]]) : M.mu[q];
            if (hi) wpm[a][2 * q] = (1.0 + mhi / M.lm[q + st[a]]) * ih2;
            if (lo) wpm[a][2 * q + 1] = (1.0 + mlo / M.lm[q - st[a]]) * ih2;
            diag += (2.0 + (mlo + mhi) / M.lm[q]) * ih2;
        }
        const std::complex<double> ms = M.rho[q] * std::complex<double>(1.0, -(M.gamma[q] / c->omega + alpha));
        D[q] = diag - om2 * ms / M.lm[q];
    }
}

std::vector<c128> fine_stencil(const eh_ctx* c, const Block& B, const std::vector<double> w[3],
                               const std::vector<std::complex<double>>& D) {
    const bool tilde = B.kind == c->dim && c->o.ap_variant == 1;
    const Dims& d = B.lev[0].d;
    const int64_t np = d.np();
    Widths wd{{1, 1, c->dim == 3 ? 1 : 0}};
    const int nst = wd.nst();
    std::vector<c128> st((size_t)nst * np, mk(0.0, 0.0));
    const int NX = 3, NY = 3;
    auto put = [&](int ox, int oy, int oz, int64_t p, double v) {
        const int o = ((oz + wd.w[2]) * NY + (oy + 1)) * NX + (ox + 1);
        st[(size_t)o * np + p] = mk(v, 0.0);
    };
    const int64_t stride[3] = {1, d.g[0], (int64_t)d.g[0] * d.g[1]};
    for (int z = 0; z < d.g[2]; ++z)
        for (int y = 0; y < d.g[1]; ++y)
            for (int x = 0; x < d.g[0]; ++x) {
                const int64_t p = ((int64_t)z * d.g[1] + y) * d.g[0] + x;
                const int P[3] = {x, y, z};
                const int o = ((0 + wd.w[2]) * NY + 1) * NX + 1;
                st[(size_t)o * np + p] = mk(D[p].real(), D[p].imag());
                for (int a = 0; a < c->dim; ++a) {
                    int e[3] = {0, 0, 0};
                    e[a] = 1;
                    const double ih2 = 1.0 / (c->h[a] * c->h[a]);
                    if (P[a] + 1 < d.g[a]) {
                        const double v = tilde ? w[a][2 * p]
                                               : (B.kind < c->dim) ? w[a][p] : w[0][p + stride[a]] * ih2;
                        put(e[0], e[1], e[2], p, -v);
                    }
                    if (P[a] >= 1) {
                        const double v = tilde ? w[a][2 * p + 1]
                                               : (B.kind < c->dim) ? w[a][p - stride[a]] : w[0][p - stride[a]] * ih2;
                        put(-e[0], -e[1], -e[2], p, -v);
                    }
                }
            }
    return st;
}

// Coarsest solve by an explicit dense inverse: Gauss-Jordan with partial
// pivoting (FP64) on [X | I], applied later as a matrix-vector product.
void build_dense(eh_ctx* c, Block& B, c128* prev, const Widths& wprev, const Dims& dc) {
    const int64_t N = dc.np();
    // the dense inverse costs 16 N^2 bytes and O(N^3) setup: keep N modest
    if (N > kDenseMax)
        throw ArgError{"coarsest grid too large for the dense direct solve (use the block-tridiagonal solve)"};
    c128* M = c->alloc<c128>((size_t)N * 2 * N);
    hipLaunchKernelGGL(k_dense_from_stencil, dim3(lin_grid(N, 64, 1 << 30)), dim3(64), 0, 0, dc, wprev, prev, M);
    HIPCHK(hipGetLastError());
    int64_t* piv = c->alloc<int64_t>(1);
    c128* pval = c->alloc<c128>(1);
    c128* mult = c->alloc<c128>(N);
    const unsigned gcols = lin_grid(2 * N);
    for (int64_t kk = 0; kk < N; ++kk) {
        hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(256), 0, 0, N, kk, M, piv, pval);
        hipLaunchKernelGGL(k_gj_swap_scale, dim3(gcols), dim3(256), 0, 0, N, kk, M, piv, pval);
        hipLaunchKernelGGL(k_gj_column, dim3(lin_grid(N)), dim3(256), 0, 0, N, kk, M, mult);
        hipLaunchKernelGGL(k_gj_eliminate, dim3(gcols, (unsigned)N), dim3(256), 0, 0, N, kk, M, mult);
    }
    HIPCHK(hipGetLastError());
    B.Nc = N;
    B.Ainv = c->alloc<c128>((size_t)N * N);
    hipLaunchKernelGGL(k_gj_extract, dim3(lin_grid(N * N, 256, 1 << 30)), dim3(256), 0, 0, N, M, B.Ainv);
    HIPCHK(hipGetLastError());
    HIPCHK(hipDeviceSynchronize());
    c->release(M);
    c->release(piv);
    c->release(pval);
    c->release(mult);
}


template <class T>
void bt_solve(eh_ctx* c, const int* kinds, int ns, const void* const* f, const int64_t* vf, void* const* out,
              const int64_t* vo, int nrhs);

// Coarsest solve by block-tridiagonal LU over groups of planes normal to the
// axis that gives the smallest groups (eh_coarse_kernels.h): every group's
// Schur complement is inverted by blocked Gauss-Jordan; the factors are
// checked by solving one system and recomputing its residual in FP64.
void build_bt(eh_ctx* c, Block& B, c128* st, const Widths& w, const Dims& d) {
    BTData& T = B.btd;
    BTPart& pt = T.pt;
    pt.d = d;
    pt.w = w;
    const int64_t N = d.np();
    int best = -1;
    double bestb = 0.0;
    for (int a = 0; a < c->dim; ++a) {
        if (w.w[a] < 1) continue;
        const double bs = (double)w.w[a] * (double)N / d.g[a];
        if (best < 0 || bs < bestb) { best = a; bestb = bs; }
    }
    if (best < 0) throw ArgError{"internal: no axis for the block-tridiagonal coarsest solve"};
    pt.ax = best;
    pt.a1 = best == 0 ? 1 : 0;
    pt.a2 = best == 2 ? 1 : 2;
    pt.gsz = w.w[best];
    pt.nb = (d.g[best] + pt.gsz - 1) / pt.gsz;
    pt.P = (int)(N / d.g[best]);
    const int nb = pt.nb;
    T.goff.assign(nb + 1, 0);
    T.offF.assign(nb, 0);
    T.offB.assign(nb, 0);
    int64_t tot = 0;
    int bmax = 0;
    for (int I = 0; I < nb; ++I) {
        const int64_t b = pt.bsize(I);
        T.goff[I + 1] = T.goff[I] + b;
        T.offF[I] = tot;
        tot += b * (b + pt.bsize(I - 1));
        bmax = std::max(bmax, (int)b);
    }
    for (int I = 0; I < nb; ++I) {
        T.offB[I] = tot;
        tot += (int64_t)pt.bsize(I) * pt.bsize(I + 1);
    }
    T.mats = c->alloc<c128>((size_t)tot);
    T.offF_d = c->alloc<int64_t>((size_t)nb);
    HIPCHK(hipMemcpy(T.offF_d, T.offF.data(), (size_t)nb * sizeof(int64_t), hipMemcpyHostToDevice));
    {
        std::vector<int> perm((size_t)N);
        for (int I = 0; I < nb; ++I)
            for (int m = 0; m < pt.bsize(I); ++m) {
                int cc[3];
                pt.coords(I, m, cc);
                perm[(size_t)(T.goff[I] + m)] = (int)pt.point(cc);
            }
        T.perm = c->alloc<int>((size_t)N);
        HIPCHK(hipMemcpy(T.perm, perm.data(), (size_t)N * sizeof(int), hipMemcpyHostToDevice));
    }
    const int bpmax = (bmax + GJB - 1) / GJB * GJB;
    c128* M = c->alloc<c128>((size_t)bpmax * bpmax);
    int* bad = c->alloc<int>(1);
    HIPCHK(hipMemset(bad, 0, sizeof(int)));
    for (int I = 0; I < nb; ++I) {
        const int b = pt.bsize(I), bprev = pt.bsize(I - 1), bnext = pt.bsize(I + 1);
        const int bp = (b + GJB - 1) / GJB * GJB;
        hipLaunchKernelGGL(k_bt_schur, dim3((unsigned)((bp + 255) / 256), (unsigned)bp), dim3(256), 0, 0, pt, st, I,
                           I > 0 ? T.mats + T.offB[I - 1] : nullptr, M, bp);
        const unsigned t64 = (unsigned)((bp + 63) / 64);
        for (int K = 0; K < bp / GJB; ++K) {
            hipLaunchKernelGGL(k_gj_diag, dim3(1), dim3(256), 0, 0, M, bp, K, bad);
            hipLaunchKernelGGL(k_gj_rowpanel, dim3(t64), dim3(256), 0, 0, M, bp, K);
            hipLaunchKernelGGL(k_gj_update, dim3(t64, t64), dim3(256), 0, 0, M, bp, K);
            hipLaunchKernelGGL(k_gj_colpanel, dim3(t64), dim3(256), 0, 0, M, bp, K);
        }
        const int ldF = b + bprev;
        hipLaunchKernelGGL(k_bt_store_inv, dim3((unsigned)((b + 255) / 256), (unsigned)b), dim3(256), 0, 0, M, bp, b,
                           T.mats + T.offF[I], ldF);
        if (I > 0)
            hipLaunchKernelGGL(k_bt_couple, dim3((unsigned)((bprev + 255) / 256), (unsigned)b), dim3(256), 0, 0, pt,
                               st, I, -1, M, bp, T.mats + T.offF[I] + b, ldF);
        if (I < nb - 1)
            hipLaunchKernelGGL(k_bt_couple, dim3((unsigned)((bnext + 255) / 256), (unsigned)b), dim3(256), 0, 0, pt,
                               st, I, +1, M, bp, T.mats + T.offB[I], bnext);
        HIPCHK(hipGetLastError());
    }
    HIPCHK(hipDeviceSynchronize());
    int hbad = 0;
    HIPCHK(hipMemcpy(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost));
    c->release(M);
    c->release(bad);
    if (hbad) throw ArgError{"coarsest level: zero pivot in the block-tridiagonal factorisation"};
    B.bt = true;
    B.Nc = N;
    // accuracy check: solve X x = f for a fixed f, recompute f - X x in FP64
    std::vector<c128> hf((size_t)N), hr((size_t)N);
    for (int64_t q = 0; q < N; ++q) hf[(size_t)q] = mk(std::sin(0.37 * (double)q + 0.1), std::cos(0.91 * (double)q));
    c128* df = c->alloc<c128>((size_t)N);
    c128* dx = c->alloc<c128>((size_t)N);
    c128* dy = c->alloc<c128>((size_t)N);
    T.y = c->alloc<c128>((size_t)N);
    HIPCHK(hipMemcpy(df, hf.data(), (size_t)N * sizeof(c128), hipMemcpyHostToDevice));
    {
        hipStream_t keep = c->s;
        c->s = nullptr;
        const int kinds[1] = {B.kind};
        const void* fp[1] = {df};
        void* xp[1] = {dx};
        const int64_t vv[1] = {N};
        bt_solve<double>(c, kinds, 1, fp, vv, xp, vv, 1);
        c->s = keep;
    }
    hipLaunchKernelGGL(k_stencil_f64, dim3(lin_grid(N, 256, 1 << 30)), dim3(256), 0, 0, d, w, st, dx, dy);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpy(hr.data(), dy, (size_t)N * sizeof(c128), hipMemcpyDeviceToHost));
    double rn = 0.0, fn = 0.0;
    for (int64_t q = 0; q < N; ++q) {
        const c128 e = hr[(size_t)q] - hf[(size_t)q];
        rn += cabs2(e);
        fn += cabs2(hf[(size_t)q]);
    }
    c->release(df);
    c->release(dx);
    c->release(dy);
    const double rel = std::sqrt(rn / fn);
    if (!(rel < 1e-8)) {
        char msg[160];
        std::snprintf(msg, sizeof msg, "coarsest level: block-tridiagonal factorisation inaccurate (relative "
                      "residual %.3g)", rel);
        throw ArgError{msg};
    }
}

// Galerkin hierarchy (FP64 on the device) and coarsest inverse.
void build_hierarchy(eh_ctx* c, Block& B, const std::vector<c128>& st0) {
    const int L = (int)B.lev.size();
    const bool f32 = c->o.mg_precision == 32;
    c128* prev = c->alloc<c128>(st0.size());
    HIPCHK(hipMemcpy(prev, st0.data(), st0.size() * sizeof(c128), hipMemcpyHostToDevice));
    Widths wprev{{1, 1, c->dim == 3 ? 1 : 0}};
    int* overflow = c->alloc<int>(1);
    HIPCHK(hipMemset(overflow, 0, sizeof(int)));
    for (int l = 1; l < L; ++l) {
        Level& Lc = B.lev[l];
        const Level& Lf = B.lev[l - 1];
        Widths wc{{0, 0, 0}};
        for (int a = 0; a < c->dim; ++a) wc.w[a] = (c->o.intergrid == 1 || (B.nodal_mask & (1 << a))) ? 1 : 2;
        Lc.w = wc;
        const int64_t npc = Lc.d.np();
        c128* cur = c->alloc<c128>((size_t)wc.nst() * npc);
        hipLaunchKernelGGL(k_galerkin, dim3(lin_grid(npc, 64, 1 << 30)), dim3(64), 0, 0, Lf.d, wprev,
                           prev, Lc.d, wc, B.nodal_mask, c->o.intergrid, cur, overflow);
        HIPCHK(hipGetLastError());
        HIPCHK(hipDeviceSynchronize());
        // store in the multigrid precision; with full weighting the shear
        // blocks stay complex symmetric, so only the offsets from the centre
        // on are kept (the others are read from the neighbours); H_p and
        // the mixed intergrid's operators in full
        Lc.half = B.kind < c->dim && c->o.intergrid == 0;
        const int ctr_full = wc.nst() / 2;
        const int64_t nst_st = Lc.nstored();
        const c128* src = Lc.half ? cur + (int64_t)ctr_full * npc : cur;
        if (f32) {
            c64* cf = c->alloc<c64>((size_t)nst_st * npc);
            hipLaunchKernelGGL((k_cast<float, double>), dim3(lin_grid(nst_st * npc)), dim3(256), 0, 0, nst_st * npc,
                               src, cf);
            HIPCHK(hipGetLastError());
            Lc.coef = cf;
        } else {
            c128* cf = c->alloc<c128>((size_t)nst_st * npc);
            HIPCHK(hipMemcpy(cf, src, (size_t)nst_st * npc * sizeof(c128), hipMemcpyDeviceToDevice));
            Lc.coef = cf;
        }
        {
            // damping / centre coefficient of the stored stencil
            const int ctr = Lc.half ? 0 : ctr_full;
            const unsigned gl = (unsigned)((npc + 255) / 256);
            if (f32) {
                Lc.dinv = c->alloc<c64>(npc);
#define EH_DI(CT) hipLaunchKernelGGL((k_dinv<float, CT>), dim3(gl), dim3(256), 0, 0, npc, (const c64*)Lc.coef, \
                                     (float)Lc.damp, (c64*)Lc.dinv)
                if (ctr == 0) EH_DI(0); else if (ctr == 12) EH_DI(12); else if (ctr == 62) EH_DI(62);
                else if (ctr == 4) EH_DI(4); else if (ctr == 13) EH_DI(13);
                else throw ArgError{"internal: unexpected stencil centre"};
#undef EH_DI
            } else {
                Lc.dinv = c->alloc<c128>(npc);
#define EH_DI(CT) hipLaunchKernelGGL((k_dinv<double, CT>), dim3(gl), dim3(256), 0, 0, npc, (const c128*)Lc.coef, \
                                     Lc.damp, (c128*)Lc.dinv)
                if (ctr == 0) EH_DI(0); else if (ctr == 12) EH_DI(12); else if (ctr == 62) EH_DI(62);
                else if (ctr == 4) EH_DI(4); else if (ctr == 13) EH_DI(13);
                else throw ArgError{"internal: unexpected stencil centre"};
#undef EH_DI
            }
            HIPCHK(hipGetLastError());
        }
        HIPCHK(hipDeviceSynchronize());
        c->release(prev);
        prev = cur;
        wprev = wc;
    }
    int ov = 0;
    HIPCHK(hipMemcpy(&ov, overflow, sizeof(int), hipMemcpyDeviceToHost));
    c->release(overflow);
    if (ov) throw ArgError{"internal: Galerkin stencil exceeded its width"};
    const Level& Lc = B.lev[L - 1];
    if (c->use_bt) build_bt(c, B, prev, wprev, Lc.d);
    else build_dense(c, B, prev, wprev, Lc.d);
    c->release(prev);
}

void ensure_mg_workspace(eh_ctx* c, int nrhs) {
    if (nrhs <= c->nrhs_cap) return;
    HIPCHK(hipStreamSynchronize(c->s));
    drop_graphs(c);
    const size_t cs = c->csize();
    for (int b = 0; b < c->nblocks; ++b)
        for (auto& L : c->blk[b].lev) {
            for (void** pp : {&L.f, &L.u, &L.t, &L.r, &L.e}) {
                c->release(*pp);
                *pp = c->alloc<char>((size_t)L.d.np() * nrhs * cs);
            }
        }
    for (int b = 0; b < c->nblocks; ++b) {
        BTData& T = c->blk[b].btd;
        if (!c->blk[b].bt) continue;
        c->release(T.y);
        T.y = c->alloc<c128>((size_t)T.pt.d.np() * nrhs);
    }
    c->nrhs_cap = nrhs;
}

void ensure_tmpT(eh_ctx* c, int64_t elems) {
    if (elems <= c->tmpT_elems) return;
    HIPCHK(hipStreamSynchronize(c->s));
    c->release(c->tmpT);
    c->tmpT = c->alloc<char>((size_t)elems * c->csize());
    c->tmpT_elems = elems;
}

// ---------------------------------------------------------------------------
// multigrid cycle (Algorithm TwoCycle, recursive; V: one call, W: two), run
// for a group of blocks at once (the shear blocks together, H_p alone)

template <class T>
GArgs<T> gbase(eh_ctx* c, const int* kinds, int ns, int l, bool coarse_dims_for_dc) {
    GArgs<T> a{};
    a.ns = ns;
    a.maxg2 = 1;
    for (int s = 0; s < ns; ++s) {
        const Block& B = c->blk[kinds[s]];
        a.kind[s] = kinds[s];
        a.d[s] = B.lev[l].d;
        if (coarse_dims_for_dc && l + 1 < (int)B.lev.size()) a.dc[s] = B.lev[l + 1].d;
        a.maxg2 = std::max(a.maxg2, a.d[s].g[2]);
        if (l == 0) {
            for (int ax = 0; ax < 3; ++ax) a.w[s][ax] = (const T*)B.fw[ax];
            a.D[s] = (const cplx<T>*)B.fD;
        } else {
            a.coef[s] = (const cplx<T>*)B.lev[l].coef;
            a.dinv[s] = (const cplx<T>*)B.lev[l].dinv;
        }
    }
    a.damp = T(c->blk[kinds[0]].lev[l].damp);
    for (int ax = 0; ax < 3; ++ax) a.ih[ax] = T(1.0 / (c->h[ax] * c->h[ax]));
    a.mixed = c->o.intergrid == 1;
    a.tilde = c->o.ap_variant == 1;
    return a;
}

// Right-hand sides per workgroup of a multigrid launch (fused leg or
// per-sweep kernel) with `tiles` workgroups per slot: the whole batch while the tiles alone give kSplitWgs workgroups or
// more (the operator in registers then serves every right-hand side);
// below that the batch is split into chunks, up to one right-hand side per
// workgroup, so that a small level runs its right-hand sides side by side
// instead of one after the other.
#ifndef EH_SPLIT_WGS
#define EH_SPLIT_WGS 4096
#endif
constexpr int kSplitWgs = EH_SPLIT_WGS;
inline int rhs_chunk(int tiles, int ns, int nrhs) {
    const int64_t wgs = (int64_t)tiles * ns;
    if (nrhs <= 1 || wgs >= kSplitWgs) return std::max(nrhs, 1);
    const int nch = (int)std::min<int64_t>(nrhs, (kSplitWgs + wgs - 1) / wgs);
    return (nrhs + nch - 1) / nch;
}

// Grid of a per-sweep kernel over the slots of a and the chunks of the
// batch; rch receives the right-hand sides per workgroup.
template <class T>
dim3 ggrid(const GArgs<T>& a, const dim3& blk, int nrhs, int& rch) {
    int gx = 1, gy = 1;
    for (int s = 0; s < a.ns; ++s) {
        gx = std::max(gx, (int)((a.d[s].g[0] + blk.x - 1) / blk.x));
        gy = std::max(gy, (int)((a.d[s].g[1] + blk.y - 1) / blk.y));
    }
    rch = rhs_chunk(gx * gy * a.maxg2, a.ns, nrhs);
    const int nch = (std::max(nrhs, 1) + rch - 1) / rch;
    return dim3((unsigned)gx, (unsigned)gy, (unsigned)(a.maxg2 * a.ns * nch));
}

// Restriction (grid = coarse level) or prolongation with correction (grid
// = fine level) for the slots of t.
template <class T>
void launch_transfer(eh_ctx* c, const GArgs<T>& t, const dim3& blk, bool restrict_to_coarse, int nrhs) {
    int rch = 1;
    if (c->dim == 3) {
        // the staged 3D transfers: tiles of 256 threads
        if (restrict_to_coarse) {
            const dim3 g = ggrid(t, dim3(RTX, RTY, 1), nrhs, rch);
            if (t.mixed) hipLaunchKernelGGL((k_grestrict3_lds<T, true>), g, dim3(256), 0, c->s, t, nrhs, rch);
            else hipLaunchKernelGGL((k_grestrict3_lds<T, false>), g, dim3(256), 0, c->s, t, nrhs, rch);
        } else {
            const dim3 g = ggrid(t, dim3(PTX, PTY, 1), nrhs, rch);
            hipLaunchKernelGGL((k_gprolong3_lds<T>), g, dim3(256), 0, c->s, t, nrhs, rch);
        }
        HIPCHK(hipGetLastError());
        return;
    }
    const dim3 g = ggrid(t, blk, nrhs, rch);
    if (restrict_to_coarse) {
        if (c->dim == 2) hipLaunchKernelGGL((k_gtransfer<T, 2, true>), g, blk, 0, c->s, t, nrhs, rch);
        else hipLaunchKernelGGL((k_gtransfer<T, 3, true>), g, blk, 0, c->s, t, nrhs, rch);
    } else {
        if (c->dim == 2) hipLaunchKernelGGL((k_gtransfer<T, 2, false>), g, blk, 0, c->s, t, nrhs, rch);
        else hipLaunchKernelGGL((k_gtransfer<T, 3, false>), g, blk, 0, c->s, t, nrhs, rch);
    }
    HIPCHK(hipGetLastError());
}

// real couplings stored per fine-level point: d edge weights (A_k), one
// cell weight (H_p), or a pair per axis (H_p from A~_p)
inline int fine_couplings(const eh_ctx* c, bool P) {
    return P ? (c->o.ap_variant == 1 ? 2 * c->dim : 1) : c->dim;
}

// block group of a launch: 0 for H_p, 1 for the shear blocks
inline int group_of(const eh_ctx* c, int kind0) { return kind0 == c->dim ? 0 : 1; }

inline dim3 shape_block(const eh_ctx* c, int group, int l, int which) {
    const int* sh = kShapes[c->shape[group][std::min(l, kMaxLevels - 1)][which]];
    return dim3((unsigned)sh[0], (unsigned)sh[1], 1);
}

// One sweep-type launch (modes of k_gfine / k_gstencil) on level l.
template <class T>
void gsweep(eh_ctx* c, GArgs<T>& a, int l, int mode, int nrhs) {
    const int kind0 = a.kind[0];
    const bool P = kind0 == c->dim;
    double by = 0.0;
    for (int s = 0; s < a.ns; ++s) {
        const Block& B = c->blk[a.kind[s]];
        const double np = (double)a.d[s].np(), cs = sizeof(cplx<T>), rs = sizeof(T);
        double coefb = l == 0 ? np * (cs + fine_couplings(c, P) * rs) : np * B.lev[l].nstored() * cs;
        double vecb = (mode == 0 || mode == 3 || mode == 5) ? 2 * np * cs : 3 * np * cs;
        if (mode == 0) coefb = np * cs;
        by += coefb + nrhs * vecb;
    }
    const int cls = l > 0 ? KC_COARSE
                          : (mode == 0 || mode == 4 || mode == 5 ? KC_FINE_FIRST
                                                                  : (mode == 1 ? KC_FINE_SWEEP : KC_FINE_RESID));
    Timed tm(c, cls, by);
    if (l == 0 && c->dim == 3 && (mode == 1 || mode == 2 || mode == 5)) {
        // the plane-staged kernel: FTX x FTY tiles of two planes, 256 threads
        int gx = 1, gy = 1;
        for (int s = 0; s < a.ns; ++s) {
            gx = std::max(gx, (a.d[s].g[0] + FTX - 1) / FTX);
            gy = std::max(gy, (a.d[s].g[1] + FTY - 1) / FTY);
        }
        const int nzb = (a.maxg2 + 1) / 2;   // plane pairs
        const int rch = rhs_chunk(gx * gy * nzb, a.ns, nrhs);
        const int nch = (std::max(nrhs, 1) + rch - 1) / rch;
        const dim3 g((unsigned)gx, (unsigned)gy, (unsigned)(nzb * a.ns * nch));
#define EH_G3(KIND)                                                                                              \
    if (mode == 1) hipLaunchKernelGGL((k_gfine3_lds<T, KIND, 1>), g, dim3(256), 0, c->s, a, nrhs, rch);          \
    else if (mode == 2) hipLaunchKernelGGL((k_gfine3_lds<T, KIND, 2>), g, dim3(256), 0, c->s, a, nrhs, rch);     \
    else hipLaunchKernelGGL((k_gfine3_lds<T, KIND, 5>), g, dim3(256), 0, c->s, a, nrhs, rch);
        if (P && a.tilde) { EH_G3(2) } else if (P) { EH_G3(1) } else { EH_G3(0) }
#undef EH_G3
        HIPCHK(hipGetLastError());
        return;
    }
    if (l > 0 && c->dim == 3 && a.mixed && (mode == 1 || mode == 2 || mode == 5)) {
        // the plane-staged 27-point kernel: STX x STY tiles of 256 threads
        const dim3 blk(STX, STY, 1);
        int rch = 1;
        const dim3 g = ggrid(a, blk, nrhs, rch);
        if (mode == 1) hipLaunchKernelGGL((k_gstencil3_lds<T, 1>), g, dim3(256), 0, c->s, a, nrhs, rch);
        else if (mode == 2) hipLaunchKernelGGL((k_gstencil3_lds<T, 2>), g, dim3(256), 0, c->s, a, nrhs, rch);
        else hipLaunchKernelGGL((k_gstencil3_lds<T, 5>), g, dim3(256), 0, c->s, a, nrhs, rch);
        HIPCHK(hipGetLastError());
        return;
    }
    const dim3 blk = shape_block(c, group_of(c, kind0), l, 0);
    int rch = 1;
    const dim3 g = ggrid(a, blk, nrhs, rch);
    if (l == 0) {
#define EH_GF(KIND, DIM, MODE) hipLaunchKernelGGL((k_gfine<T, KIND, DIM, MODE>), g, blk, 0, c->s, a, nrhs, rch)
#define EH_GF_M(KIND, DIM)                      \
    switch (mode) {                             \
        case 0: EH_GF(KIND, DIM, 0); break;     \
        case 1: EH_GF(KIND, DIM, 1); break;     \
        case 2: EH_GF(KIND, DIM, 2); break;     \
        case 3: EH_GF(KIND, DIM, 3); break;     \
        case 4: EH_GF(KIND, DIM, 4); break;     \
        default: EH_GF(KIND, DIM, 5); break;    \
    }
        if (c->dim == 2) {
            if (P && a.tilde) { EH_GF_M(2, 2) } else if (P) { EH_GF_M(1, 2) } else { EH_GF_M(0, 2) }
        } else {
            if (P && a.tilde) { EH_GF_M(2, 3) } else if (P) { EH_GF_M(1, 3) } else { EH_GF_M(0, 3) }
        }
#undef EH_GF_M
#undef EH_GF
    } else {
#define EH_GS(DIM, MODE)                                                                   \
    if (a.mixed) hipLaunchKernelGGL((k_gstencil<T, DIM, MODE, true>), g, blk, 0, c->s, a, nrhs, rch);  \
    else hipLaunchKernelGGL((k_gstencil<T, DIM, MODE, false>), g, blk, 0, c->s, a, nrhs, rch)
#define EH_GS_M(DIM)                        \
    switch (mode) {                         \
        case 0: EH_GS(DIM, 0); break;       \
        case 1: EH_GS(DIM, 1); break;       \
        case 2: EH_GS(DIM, 2); break;       \
        case 3: EH_GS(DIM, 3); break;       \
        case 4: EH_GS(DIM, 4); break;       \
        default: EH_GS(DIM, 5); break;      \
    }
        if (c->dim == 2) { EH_GS_M(2) } else { EH_GS_M(3) }
#undef EH_GS_M
#undef EH_GS
    }
    HIPCHK(hipGetLastError());
}

template <class T>
void gcopy(eh_ctx* c, int ns, const void* const* src, const int64_t* vs, void* const* dst, const int64_t* vd,
           const int64_t* np, int nrhs) {
    for (int s = 0; s < ns; ++s) {
        hipLaunchKernelGGL((k_copy_strided<cplx<T>>), dim3(lin_grid(np[s], 256, 4096), nrhs), dim3(256), 0, c->s,
                           np[s], nrhs, (const cplx<T>*)src[s], vs[s], (cplx<T>*)dst[s], vd[s]);
        HIPCHK(hipGetLastError());
    }
}

template <class T>
void gcycle(eh_ctx* c, const int* kinds, int ns, int l, const void* const* f, const int64_t* vf,
            void* const* out, const int64_t* vo, bool guess, int nrhs);

// Coarsest solve e = X_c^-1 f for the blocks kinds[0..ns) by the block-
// tridiagonal factors: every group's S_I^-1 f_I in one launch, then the
// forward sweep over the groups adding -S_I^-1 L_I y_{I-1}, then the back
// sweep adding B_I x_{I+1}, one launch per group step for all blocks of
// the launch (a block with fewer groups idles in the last steps; the first
// forward step has nothing to add).  Right-hand sides in chunks of up to 8
// per workgroup (the steps of batches up to 4: one), each matrix row read
// once per chunk.
template <class T>
void bt_solve(eh_ctx* c, const int* kinds, int ns, const void* const* f, const int64_t* vf, void* const* out,
              const int64_t* vo, int nrhs) {
    if (ns > BT_MAXS) throw ArgError{"internal: too many blocks for one block-tridiagonal launch"};
    if (nrhs < 1) return;
    const int RB = nrhs >= 5 ? 8 : nrhs >= 3 ? 4 : nrhs;
    const unsigned chunks = (unsigned)((nrhs + RB - 1) / RB);
    int maxnb = 0, maxb0 = 1;
    BTAll<T> fa{};
    fa.ns = ns;
    fa.nrhs = nrhs;
    double fby = 0.0;
    for (int s = 0; s < ns; ++s) {
        const BTData& bd = c->blk[kinds[s]].btd;
        const BTPart& pt = bd.pt;
        maxnb = std::max(maxnb, pt.nb);
        fa.N[s] = (int)pt.d.np();
        fa.b0[s] = pt.bsize(0);
        fa.nb[s] = pt.nb;
        fa.mats[s] = bd.mats;
        fa.offF[s] = bd.offF_d;
        fa.perm[s] = bd.perm;
        fa.y[s] = bd.y;
        fa.f[s] = (const cplx<T>*)f[s];
        fa.vf[s] = vf[s];
        maxb0 = std::max(maxb0, fa.b0[s]);
        // algorithmic bytes: the S_I^-1 blocks once per chunk, f read, y written
        for (int I = 0; I < pt.nb; ++I) fby += (double)pt.bsize(I) * pt.bsize(I) * sizeof(c128) * chunks;
        fby += (double)fa.N[s] * nrhs * (sizeof(cplx<T>) + sizeof(c128));
    }
    {
        Timed tm(c, KC_DENSE, fby);
        const dim3 g((unsigned)((maxb0 + BT_RW - 1) / BT_RW), (unsigned)(maxnb * ns), chunks);
        if (RB == 8) hipLaunchKernelGGL((k_bt_fpart<T, 8>), g, dim3(256), 0, c->s, fa);
        else if (RB == 4) hipLaunchKernelGGL((k_bt_fpart<T, 4>), g, dim3(256), 0, c->s, fa);
        else if (RB == 2) hipLaunchKernelGGL((k_bt_fpart<T, 2>), g, dim3(256), 0, c->s, fa);
        else hipLaunchKernelGGL((k_bt_fpart<T, 1>), g, dim3(256), 0, c->s, fa);
        HIPCHK(hipGetLastError());
    }
    // The sweep steps are latency-bound: up to 4 right-hand sides, one per
    // workgroup (a shorter chain of work per workgroup, the rows re-read
    // from the caches) beats reading the rows once for the batch (192^3 x 4:
    // 111 -> 90 ms per solve).  Algorithmic bytes of one step: the matrix
    // rows once per chunk of up to 8 right-hand sides, the neighbour's
    // vector entries read, this group's read and written (and e written in
    // the back sweep).
    const int RBc = nrhs <= 4 ? 1 : RB;
    const unsigned chunksc = (unsigned)((nrhs + RBc - 1) / RBc);
    auto step_bytes = [&](bool fwd, const BTStep<T>& a) {
        double by = 0.0;
        for (int s = 0; s < ns; ++s) {
            const double b = a.b[s], bo = a.bo[s];
            by += b * bo * sizeof(c128) * chunks;
            by += nrhs * (bo * sizeof(c128) + b * (2.0 * sizeof(c128) + (fwd ? 0.0 : (double)sizeof(cplx<T>))));
        }
        return by;
    };
    auto launch = [&](bool fwd, const BTStep<T>& a, int maxb) {
        Timed tm(c, KC_DENSE, step_bytes(fwd, a));
        const dim3 g((unsigned)((std::max(maxb, 1) + BT_RW - 1) / BT_RW), (unsigned)ns, chunksc);
#define EH_BT(RBV)                                                                          \
    if (fwd) hipLaunchKernelGGL((k_bt_chain<T, RBV, false>), g, dim3(256), 0, c->s, a);     \
    else hipLaunchKernelGGL((k_bt_chain<T, RBV, true>), g, dim3(256), 0, c->s, a);
        if (RBc == 8) { EH_BT(8) } else if (RBc == 4) { EH_BT(4) } else if (RBc == 2) { EH_BT(2) } else { EH_BT(1) }
#undef EH_BT
        HIPCHK(hipGetLastError());
    };
    for (int pass = 0; pass < 2; ++pass) {
        const bool fwd = pass == 0;
        for (int k = fwd ? 1 : 0; k < maxnb; ++k) {
            BTStep<T> a{};
            a.ns = ns;
            a.nrhs = nrhs;
            int maxb = 0;
            for (int s = 0; s < ns; ++s) {
                const BTData& bd = c->blk[kinds[s]].btd;
                const BTPart& pt = bd.pt;
                a.ldy[s] = pt.d.np();
                a.e[s] = (cplx<T>*)out[s];
                a.ve[s] = vo[s];
                const int I = fwd ? k : pt.nb - 1 - k;
                if (k >= pt.nb) {
                    a.b[s] = 0; a.bo[s] = 0; a.lda[s] = 0;
                    a.mat[s] = bd.mats; a.perm[s] = bd.perm; a.y[s] = bd.y; a.yo[s] = bd.y;
                    continue;
                }
                const int J = fwd ? I - 1 : I + 1;
                a.b[s] = pt.bsize(I);
                a.bo[s] = pt.bsize(J);
                // forward: the coupling columns of F_I (after its b_I columns of S_I^-1)
                a.lda[s] = fwd ? a.b[s] + a.bo[s] : a.bo[s];
                a.mat[s] = bd.mats + (fwd ? bd.offF[I] + a.b[s] : bd.offB[I]);
                a.perm[s] = bd.perm + bd.goff[I];
                a.y[s] = bd.y + bd.goff[I];
                a.yo[s] = bd.y + ((J >= 0 && J < pt.nb) ? bd.goff[J] : 0);
                maxb = std::max(maxb, a.b[s]);
            }
            launch(fwd, a, maxb);
        }
    }
}

// The fused legs cover 2D V(1, nu2) cycles started from a zero guess.
// (The legs index a level's points with 32-bit integers.)
inline bool fused_cycle(const eh_ctx* c, bool guess) {
    return c->o.fused && c->dim == 2 && c->o.cycle == 0 && c->o.nu_pre == 1 &&
           (c->o.nu_post == 1 || c->o.nu_post == 2) && !guess && (c->n[0] + 1) * (c->n[1] + 1) < (1LL << 31);
}

// One level of a V(1, nu2) cycle from a zero guess with the fused legs:
// f_{l+1} = R (f - X w D^-1 f), the cycle on level l+1, then
// out = S^nu2 (w D^-1 f + P e_{l+1}).

// Fused down leg on level l with tile configuration cfg: a.d / a.dc = levels
// l / l+1, a.f = f_l, a.out = f_{l+1}.
template <class T>
void launch_fdown(eh_ctx* c, const GArgs<T>& a, int l, int cfg, int nrhs) {
    const FCfg k = kFDown[cfg];
    int gx = 1, gy = 1;
    for (int s = 0; s < a.ns; ++s) {
        gx = std::max(gx, (a.dc[s].g[0] + k.x - 1) / k.x);
        gy = std::max(gy, (a.dc[s].g[1] + k.y - 1) / k.y);
    }
    const int rch = rhs_chunk(gx * gy, a.ns, nrhs);
    const int nch = (std::max(nrhs, 1) + rch - 1) / rch;
    const dim3 g((unsigned)gx, (unsigned)gy, (unsigned)(a.ns * nch)), blk((unsigned)k.threads);
#define EH_LFD(CF)                                                                               \
    if (l == 0) hipLaunchKernelGGL((k_fdown<T, true, CF>), g, blk, 0, c->s, a, nrhs, rch);       \
    else hipLaunchKernelGGL((k_fdown<T, false, CF>), g, blk, 0, c->s, a, nrhs, rch);
    switch (cfg) {
        case 0: EH_LFD(0) break;
        case 1: EH_LFD(1) break;
        case 2: EH_LFD(2) break;
        default: EH_LFD(3) break;
    }
#undef EH_LFD
    HIPCHK(hipGetLastError());
}

// Fused up leg on level l: a.f = f_l, a.u = e_{l+1}, a.out = e_l.
template <class T>
void launch_fup(eh_ctx* c, const GArgs<T>& a, int l, int cfg, int nrhs) {
    const FCfg k = kFUp[cfg];
    int gx = 1, gy = 1;
    for (int s = 0; s < a.ns; ++s) {
        gx = std::max(gx, (a.d[s].g[0] + k.x - 1) / k.x);
        gy = std::max(gy, (a.d[s].g[1] + k.y - 1) / k.y);
    }
    const int rch = rhs_chunk(gx * gy, a.ns, nrhs);
    const int nch = (std::max(nrhs, 1) + rch - 1) / rch;
    const dim3 g((unsigned)gx, (unsigned)gy, (unsigned)(a.ns * nch)), blk((unsigned)k.threads);
    const bool two = c->o.nu_post == 2;
#define EH_LFU(CF)                                                                                    \
    if (l == 0) {                                                                                     \
        if (two) hipLaunchKernelGGL((k_fup<T, true, 2, CF>), g, blk, 0, c->s, a, nrhs, rch);          \
        else hipLaunchKernelGGL((k_fup<T, true, 1, CF>), g, blk, 0, c->s, a, nrhs, rch);              \
    } else {                                                                                          \
        if (two) hipLaunchKernelGGL((k_fup<T, false, 2, CF>), g, blk, 0, c->s, a, nrhs, rch);         \
        else hipLaunchKernelGGL((k_fup<T, false, 1, CF>), g, blk, 0, c->s, a, nrhs, rch);             \
    }
    switch (cfg) {
        case 0: EH_LFU(0) break;
        case 1: EH_LFU(1) break;
        case 2: EH_LFU(2) break;
        default: EH_LFU(3) break;
    }
#undef EH_LFU
    HIPCHK(hipGetLastError());
}

template <class T>
void fused_level(eh_ctx* c, const int* kinds, int ns, int l, const void* const* f, const int64_t* vf,
                 void* const* out, const int64_t* vo, int nrhs) {
    const bool P = kinds[0] == c->dim;
    const int grp = group_of(c, kinds[0]);
    const int lt = std::min(l, kMaxLevels - 1);
    GArgs<T> a = gbase<T>(c, kinds, ns, l, true);
    const void* cf[GMAX];
    void* ce[GMAX];
    int64_t vcv[GMAX];
    double cbytes = 0.0, vdown = 0.0, vup = 0.0;
    const double cs = sizeof(cplx<T>), rs = sizeof(T);
    for (int s = 0; s < ns; ++s) {
        const Block& B = c->blk[kinds[s]];
        const Level& Lv = B.lev[l];
        const Level& Cv = B.lev[l + 1];
        const double np = (double)Lv.d.np(), npc = (double)Cv.d.np();
        cbytes += l == 0 ? np * (cs + fine_couplings(c, P) * rs) : np * (Lv.nstored() + 1) * cs;
        vdown += (np + npc) * cs;
        vup += (2 * np + npc) * cs;
        cf[s] = Cv.f; ce[s] = Cv.e; vcv[s] = Cv.d.np();
    }
    {
        for (int s = 0; s < ns; ++s) {
            a.f[s] = (const cplx<T>*)f[s];
            a.vf[s] = vf[s];
            a.out[s] = (cplx<T>*)cf[s];
            a.vo[s] = vcv[s];
        }
        Timed tm(c, l == 0 ? KC_FINE_DOWN : KC_COARSE_DOWN, cbytes + nrhs * vdown);
        launch_fdown<T>(c, a, l, c->fcfg[grp][lt][0], nrhs);
    }
    gcycle<T>(c, kinds, ns, l + 1, cf, vcv, ce, vcv, false, nrhs);
    {
        for (int s = 0; s < ns; ++s) {
            a.f[s] = (const cplx<T>*)f[s];
            a.vf[s] = vf[s];
            a.u[s] = (const cplx<T>*)ce[s];
            a.vu[s] = vcv[s];
            a.out[s] = (cplx<T>*)out[s];
            a.vo[s] = vo[s];
        }
        Timed tm(c, l == 0 ? KC_FINE_UP : KC_COARSE_UP, cbytes + nrhs * vup);
        launch_fup<T>(c, a, l, c->fcfg[grp][lt][1], nrhs);
    }
}

// One cycle on level l for X_l e = f, for the blocks kinds[0..ns).  f[s]
// has stride vf[s]; the result goes to out[s] (stride vo[s]).  With guess,
// out[s] holds the initial guess.
template <class T>
void gcycle(eh_ctx* c, const int* kinds, int ns, int l, const void* const* f, const int64_t* vf,
            void* const* out, const int64_t* vo, bool guess, int nrhs) {
    const int Lv = (int)c->blk[kinds[0]].lev.size();
    Level* L[GMAX];
    int64_t np[GMAX];
    for (int s = 0; s < ns; ++s) { L[s] = &c->blk[kinds[s]].lev[l]; np[s] = L[s]->d.np(); }
    if (l == Lv - 1 && c->use_bt) {
        bt_solve<T>(c, kinds, ns, f, vf, out, vo, nrhs);
        return;
    }
    if (l == Lv - 1) {
        GArgs<T> a = gbase<T>(c, kinds, ns, l, false);
        DenseArgs da{};
        da.ns = ns;
        int Nmax = 1;
        for (int s = 0; s < ns; ++s) {
            const Block& B = c->blk[kinds[s]];
            da.N[s] = (int)B.Nc;
            da.Ainv[s] = B.Ainv;
            Nmax = std::max(Nmax, da.N[s]);
        }
        int r = 0;
        while (r < nrhs) {
            // one timed launch per chunk: the inverse once, the chunk's vectors
            const int rb = nrhs - r >= 8 ? 8 : nrhs - r >= 4 ? 4 : nrhs - r >= 2 ? 2 : 1;
            double by = 0.0;
            for (int s = 0; s < ns; ++s) {
                const double N = (double)c->blk[kinds[s]].Nc;
                by += N * N * sizeof(c128) + 2.0 * N * rb * sizeof(cplx<T>);
            }
            Timed tm(c, KC_DENSE, by);
            for (int s = 0; s < ns; ++s) {
                a.f[s] = (const cplx<T>*)f[s] + (int64_t)r * vf[s];
                a.out[s] = (cplx<T>*)out[s] + (int64_t)r * vo[s];
                a.vf[s] = vf[s];
                a.vo[s] = vo[s];
            }
            const dim3 g((unsigned)Nmax, (unsigned)ns);        // one row per workgroup
            const int left = nrhs - r;
            if (left >= 8) { hipLaunchKernelGGL((k_gdense<T, 8>), g, dim3(256), 0, c->s, da, a); r += 8; }
            else if (left >= 4) { hipLaunchKernelGGL((k_gdense<T, 4>), g, dim3(256), 0, c->s, da, a); r += 4; }
            else if (left >= 2) { hipLaunchKernelGGL((k_gdense<T, 2>), g, dim3(256), 0, c->s, da, a); r += 2; }
            else { hipLaunchKernelGGL((k_gdense<T, 1>), g, dim3(256), 0, c->s, da, a); r += 1; }
            HIPCHK(hipGetLastError());
        }
        return;
    }
    const int nu1 = c->o.nu_pre, nu2 = c->o.nu_post;
    if (fused_cycle(c, guess)) {
        fused_level<T>(c, kinds, ns, l, f, vf, out, vo, nrhs);
        return;
    }
    const void* cur[GMAX];
    int64_t vcur[GMAX];
    int nb = 0;   // next internal buffer: 0 -> u, 1 -> t
    auto buf = [&](int s, int which) -> void* { return which == 0 ? L[s]->u : L[s]->t; };
    GArgs<T> a = gbase<T>(c, kinds, ns, l, false);
    bool have_resid = false;
    auto sweep = [&](int mode, bool to_out_last) {
        // one sweep from cur into a fresh buffer (or into out)
        void* dst[GMAX];
        int64_t vd[GMAX];
        bool use_out = to_out_last;
        for (int s = 0; s < ns; ++s) if (cur[s] == out[s]) use_out = false;
        int which = nb;
        if (!use_out) {
            bool clash = false;
            for (int s = 0; s < ns; ++s) if (buf(s, which) == cur[s]) clash = true;
            if (clash) which ^= 1;
            nb = which ^ 1;
        }
        for (int s = 0; s < ns; ++s) {
            dst[s] = use_out ? out[s] : buf(s, which);
            vd[s] = use_out ? vo[s] : np[s];
            a.f[s] = (const cplx<T>*)f[s];
            a.vf[s] = vf[s];
            a.u[s] = (const cplx<T>*)cur[s];
            a.vu[s] = vcur[s];
            a.out[s] = (cplx<T>*)dst[s];
            a.vo[s] = vd[s];
        }
        gsweep<T>(c, a, l, mode, nrhs);
        for (int s = 0; s < ns; ++s) { cur[s] = dst[s]; vcur[s] = vd[s]; }
    };
    if (guess) {
        for (int s = 0; s < ns; ++s) { cur[s] = out[s]; vcur[s] = vo[s]; }
        for (int t = 0; t < nu1; ++t) sweep(1, false);
    } else if (nu1 == 1) {
        // first sweep fused with the residual
        for (int s = 0; s < ns; ++s) {
            a.f[s] = (const cplx<T>*)f[s];
            a.vf[s] = vf[s];
            a.out[s] = (cplx<T>*)L[s]->u;
            a.vo[s] = np[s];
            a.out2[s] = (cplx<T>*)L[s]->r;
            a.vo2[s] = np[s];
        }
        gsweep<T>(c, a, l, 4, nrhs);
        for (int s = 0; s < ns; ++s) { cur[s] = L[s]->u; vcur[s] = np[s]; }
        nb = 1;
        have_resid = true;
    } else if (nu1 > 1) {
        // the first two sweeps from zero in one pass
        for (int s = 0; s < ns; ++s) {
            a.f[s] = (const cplx<T>*)f[s];
            a.vf[s] = vf[s];
            a.out[s] = (cplx<T>*)L[s]->u;
            a.vo[s] = np[s];
        }
        gsweep<T>(c, a, l, 5, nrhs);
        for (int s = 0; s < ns; ++s) { cur[s] = L[s]->u; vcur[s] = np[s]; }
        nb = 1;
        for (int t = 2; t < nu1; ++t) sweep(1, false);
    } else {
        for (int s = 0; s < ns; ++s) {
            hipLaunchKernelGGL((k_fill<cplx<T>>), dim3(lin_grid(np[s] * nrhs, 256, 4096)), dim3(256), 0, c->s,
                               np[s] * nrhs, (cplx<T>*)L[s]->u, czero<T>());
            HIPCHK(hipGetLastError());
            cur[s] = L[s]->u; vcur[s] = np[s];
        }
        nb = 1;
    }
    if (!have_resid) {
        for (int s = 0; s < ns; ++s) {
            a.f[s] = (const cplx<T>*)f[s];
            a.vf[s] = vf[s];
            a.u[s] = (const cplx<T>*)cur[s];
            a.vu[s] = vcur[s];
            a.out[s] = (cplx<T>*)L[s]->r;
            a.vo[s] = np[s];
        }
        gsweep<T>(c, a, l, 2, nrhs);
    }
    // restriction onto level l+1 (kernel grid = coarse; dc[] = fine grid)
    Level* C[GMAX];
    int64_t npc[GMAX];
    const void* cf[GMAX];
    void* ce[GMAX];
    int64_t vcv[GMAX];
    {
        GArgs<T> t = gbase<T>(c, kinds, ns, l + 1, false);
        double by = 0.0;
        for (int s = 0; s < ns; ++s) {
            C[s] = &c->blk[kinds[s]].lev[l + 1];
            npc[s] = C[s]->d.np();
            t.dc[s] = L[s]->d;
            t.f[s] = (const cplx<T>*)L[s]->r;
            t.vf[s] = np[s];
            t.out[s] = (cplx<T>*)C[s]->f;
            t.vo[s] = npc[s];
            cf[s] = C[s]->f; ce[s] = C[s]->e; vcv[s] = npc[s];
            by += (double)(np[s] + npc[s]) * nrhs * sizeof(cplx<T>);
        }
        Timed tm(c, KC_RESTRICT, by);
        const dim3 blk = shape_block(c, group_of(c, kinds[0]), l, 1);
        launch_transfer<T>(c, t, blk, true, nrhs);
        HIPCHK(hipGetLastError());
    }
    // W: two calls on level l+1, except when it is the coarsest level, whose
    // direct solve would give the same result again
    const int ncalls = (c->o.cycle == 1 && l + 2 < Lv) ? 2 : 1;
    for (int t = 0; t < ncalls; ++t) gcycle<T>(c, kinds, ns, l + 1, cf, vcv, ce, vcv, t > 0, nrhs);
    // prolongation and correction, in place on cur (elementwise)
    {
        GArgs<T> t = gbase<T>(c, kinds, ns, l, true);
        double by = 0.0;
        for (int s = 0; s < ns; ++s) {
            t.f[s] = (const cplx<T>*)C[s]->e;
            t.vf[s] = npc[s];
            t.out[s] = (cplx<T>*)cur[s];
            t.vo[s] = vcur[s];
            by += (double)(2 * np[s] + npc[s]) * nrhs * sizeof(cplx<T>);
        }
        Timed tm(c, KC_PROLONG, by);
        const dim3 blk = shape_block(c, group_of(c, kinds[0]), l, 2);
        launch_transfer<T>(c, t, blk, false, nrhs);
        HIPCHK(hipGetLastError());
    }
    for (int t = 0; t < nu2; ++t) sweep(1, t == nu2 - 1);
    bool need_copy = false;
    for (int s = 0; s < ns; ++s) if (cur[s] != out[s]) need_copy = true;
    if (need_copy) gcopy<T>(c, ns, cur, vcur, out, vo, np, nrhs);
}

// ---------------------------------------------------------------------------
// launch-shape autotuner

std::string tune_signature(const eh_ctx* c, int nrhs) {
    char buf[256];
    std::snprintf(buf, sizeof(buf), "d%d n%lldx%lldx%lld L%d p%d i%d r%d f%d n%d a%d", c->dim,
                  (long long)c->n[0], (long long)c->n[1], (long long)c->n[2], c->o.levels, c->o.mg_precision,
                  c->o.intergrid, nrhs, c->o.fused, c->o.nu_post, c->o.ap_variant);
    return buf;
}

bool tune_cache_load(eh_ctx* c, const std::string& sig) {
    const char* path = std::getenv("EH_TUNE_CACHE");
    if (!path) return false;
    FILE* fp = std::fopen(path, "r");
    if (!fp) return false;
    char line[4096];
    bool found = false;
    while (std::fgets(line, sizeof(line), fp)) {
        std::string ln(line);
        const size_t bar = ln.find(" | ");
        if (bar == std::string::npos || ln.substr(0, bar) != sig) continue;
        const char* q = ln.c_str() + bar + 3;
        int vals[2 * kMaxLevels * 5];
        int cnt = 0;
        char* end = nullptr;
        while (cnt < 2 * kMaxLevels * 5) {
            long v = std::strtol(q, &end, 10);
            if (end == q) break;
            vals[cnt++] = (int)v;
            q = end;
        }
        const int nsh = 2 * c->o.levels * 3;
        if (cnt != nsh + 2 * c->o.levels * 2) continue;
        bool ok = true;
        for (int t = 0; t < cnt; ++t)
            if (vals[t] < 0 || vals[t] >= (t < nsh ? kNumShapes : kFCfgs)) ok = false;
        if (!ok) continue;
        int t = 0;
        for (int g = 0; g < 2; ++g)
            for (int l = 0; l < c->o.levels; ++l)
                for (int w = 0; w < 3; ++w) c->shape[g][l][w] = vals[t++];
        for (int g = 0; g < 2; ++g)
            for (int l = 0; l < c->o.levels; ++l)
                for (int w = 0; w < 2; ++w) c->fcfg[g][l][w] = vals[t++];
        found = true;
    }
    std::fclose(fp);
    return found;
}

void tune_cache_store(const eh_ctx* c, const std::string& sig) {
    const char* path = std::getenv("EH_TUNE_CACHE");
    if (!path) return;
    FILE* fp = std::fopen(path, "a");
    if (!fp) return;
    std::fprintf(fp, "%s |", sig.c_str());
    for (int g = 0; g < 2; ++g)
        for (int l = 0; l < c->o.levels; ++l)
            for (int w = 0; w < 3; ++w) std::fprintf(fp, " %d", c->shape[g][l][w]);
    for (int g = 0; g < 2; ++g)
        for (int l = 0; l < c->o.levels; ++l)
            for (int w = 0; w < 2; ++w) std::fprintf(fp, " %d", c->fcfg[g][l][w]);
    std::fprintf(fp, "\n");
    std::fclose(fp);
}

// Time `launch` (one launch per call) for every shape; return the fastest.
template <class F>
int pick_shape(eh_ctx* c, F launch) {
    hipEvent_t a = take_event(c), b = take_event(c);
    int best = 0;
    float best_ms = 1e30f;
    for (int sh = 0; sh < kNumShapes; ++sh) {
        const dim3 blk((unsigned)kShapes[sh][0], (unsigned)kShapes[sh][1], 1);
        launch(blk);                                   // warm-up
        HIPCHK(hipEventRecord(a, c->s));
        for (int rep = 0; rep < 3; ++rep) launch(blk);
        HIPCHK(hipEventRecord(b, c->s));
        HIPCHK(hipEventSynchronize(b));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, a, b));
        if (ms < best_ms) { best_ms = ms; best = sh; }
    }
    c->event_pool.push_back(a);
    c->event_pool.push_back(b);
    return best;
}

// Time `launch(cfg)` for every fused-leg tile configuration; return the
// one with the smallest median.  Candidates alternate launch by launch, so
// each timed launch follows a different kernel, as in a cycle: on small
// levels a kernel's time includes fetching its instructions into a cold
// cache, and single launches of a few microseconds are noisy.
template <class F>
int pick_cfg(eh_ctx* c, F launch) {
    constexpr int kReps = 7;
    hipEvent_t ev[2 * kFCfgs];
    for (auto& e : ev) e = take_event(c);
    float t[kFCfgs][kReps] = {};
    for (int cf = 0; cf < kFCfgs; ++cf) launch(cf);   // warm-up
    for (int rep = 0; rep < kReps; ++rep) {
        for (int cf = 0; cf < kFCfgs; ++cf) {
            HIPCHK(hipEventRecord(ev[2 * cf], c->s));
            launch(cf);
            HIPCHK(hipEventRecord(ev[2 * cf + 1], c->s));
        }
        HIPCHK(hipEventSynchronize(ev[2 * kFCfgs - 1]));
        for (int cf = 0; cf < kFCfgs; ++cf) HIPCHK(hipEventElapsedTime(&t[cf][rep], ev[2 * cf], ev[2 * cf + 1]));
    }
    for (auto e : ev) c->event_pool.push_back(e);
    int best = 0;
    float best_ms = 1e30f;
    for (int cf = 0; cf < kFCfgs; ++cf) {
        std::sort(t[cf], t[cf] + kReps);
        if (t[cf][kReps / 2] < best_ms) { best_ms = t[cf][kReps / 2]; best = cf; }
    }
    return best;
}

// Pick the workgroup shape of the sweep, restriction and prolongation
// kernels of every level and block group for this batch size, timing each
// candidate on the level's own buffers.  Arithmetic per point does not
// depend on the shape, so results are unchanged bitwise.
template <class T>
void maybe_autotune(eh_ctx* c, int nrhs) {
    if (!c->o.autotune || c->tuned_nrhs == nrhs) return;
    ensure_mg_workspace(c, nrhs);
    drop_graphs(c);
    const std::string sig = tune_signature(c, nrhs);
    if (tune_cache_load(c, sig)) { c->tuned_nrhs = nrhs; return; }
    const unsigned saved_mask = c->timer_mask;
    c->timer_mask = 0;
    const int L = c->o.levels;
    for (int g = 0; g < 2; ++g) {
        int kinds[GMAX];
        int ns = 0;
        if (g == 0) kinds[ns++] = c->dim;
        else for (int k = 0; k < c->dim; ++k) kinds[ns++] = k;
        if (fused_cycle(c, false)) {
            // the fused legs are the only level kernels at this batch size
            for (int l = 0; l < L; ++l)
                for (int s = 0; s < ns; ++s) {
                    Level& Lv = c->blk[kinds[s]].lev[l];
                    const int64_t tot = Lv.d.np() * nrhs;
                    for (void* p : {Lv.f, Lv.u, Lv.e})
                        hipLaunchKernelGGL((k_fill<cplx<T>>), dim3(lin_grid(tot, 256, 4096)), dim3(256), 0, c->s,
                                           tot, (cplx<T>*)p, mk<T>(T(0.5), T(-0.25)));
                }
            HIPCHK(hipGetLastError());
            for (int l = 0; l + 1 < L; ++l) {
                GArgs<T> a = gbase<T>(c, kinds, ns, l, true);
                for (int s = 0; s < ns; ++s) {
                    Level& Lv = c->blk[kinds[s]].lev[l];
                    Level& Cv = c->blk[kinds[s]].lev[l + 1];
                    a.f[s] = (const cplx<T>*)Lv.f; a.vf[s] = Lv.d.np();
                    a.out[s] = (cplx<T>*)Cv.f; a.vo[s] = Cv.d.np();
                }
                c->fcfg[g][l][0] = pick_cfg(c, [&](int cf) { launch_fdown<T>(c, a, l, cf, nrhs); });
                for (int s = 0; s < ns; ++s) {
                    Level& Lv = c->blk[kinds[s]].lev[l];
                    Level& Cv = c->blk[kinds[s]].lev[l + 1];
                    a.u[s] = (const cplx<T>*)Cv.e; a.vu[s] = Cv.d.np();
                    a.out[s] = (cplx<T>*)Lv.u; a.vo[s] = Lv.d.np();
                }
                c->fcfg[g][l][1] = pick_cfg(c, [&](int cf) { launch_fup<T>(c, a, l, cf, nrhs); });
            }
            continue;
        }
        for (int l = 0; l < L; ++l) {
            for (int s = 0; s < ns; ++s) {
                Level& Lv = c->blk[kinds[s]].lev[l];
                const int64_t tot = Lv.d.np() * nrhs;
                for (void* p : {Lv.f, Lv.u, Lv.t, Lv.r, Lv.e})
                    hipLaunchKernelGGL((k_fill<cplx<T>>), dim3(lin_grid(tot, 256, 4096)), dim3(256), 0, c->s, tot,
                                       (cplx<T>*)p, mk<T>(T(0.5), T(-0.25)));
            }
            HIPCHK(hipGetLastError());
            if (l == L - 1) break;
            // sweeps
            GArgs<T> a = gbase<T>(c, kinds, ns, l, false);
            for (int s = 0; s < ns; ++s) {
                Level& Lv = c->blk[kinds[s]].lev[l];
                a.f[s] = (const cplx<T>*)Lv.f; a.vf[s] = Lv.d.np();
                a.u[s] = (const cplx<T>*)Lv.u; a.vu[s] = Lv.d.np();
                a.out[s] = (cplx<T>*)Lv.t; a.vo[s] = Lv.d.np();
            }
            c->shape[g][l][0] = pick_shape(c, [&](const dim3& blk) {
                const int keep = c->shape[g][l][0];
                for (int sh = 0; sh < kNumShapes; ++sh)
                    if ((int)blk.x == kShapes[sh][0] && (int)blk.y == kShapes[sh][1]) c->shape[g][l][0] = sh;
                gsweep<T>(c, a, l, 1, nrhs);
                c->shape[g][l][0] = keep;
            });
            // restriction (grid = level l+1) and prolongation (grid = level l)
            GArgs<T> rt = gbase<T>(c, kinds, ns, l + 1, false);
            GArgs<T> pt = gbase<T>(c, kinds, ns, l, true);
            for (int s = 0; s < ns; ++s) {
                Level& Lv = c->blk[kinds[s]].lev[l];
                Level& Cv = c->blk[kinds[s]].lev[l + 1];
                rt.dc[s] = Lv.d;
                rt.f[s] = (const cplx<T>*)Lv.r; rt.vf[s] = Lv.d.np();
                rt.out[s] = (cplx<T>*)Cv.f; rt.vo[s] = Cv.d.np();
                pt.f[s] = (const cplx<T>*)Cv.e; pt.vf[s] = Cv.d.np();
                pt.out[s] = (cplx<T>*)Lv.u; pt.vo[s] = Lv.d.np();
            }
            c->shape[g][l][1] = pick_shape(c, [&](const dim3& blk) {
                launch_transfer<T>(c, rt, blk, true, nrhs);
                HIPCHK(hipGetLastError());
            });
            c->shape[g][l][2] = pick_shape(c, [&](const dim3& blk) {
                launch_transfer<T>(c, pt, blk, false, nrhs);
                HIPCHK(hipGetLastError());
            });
        }
    }
    HIPCHK(hipStreamSynchronize(c->s));
    c->timer_mask = saved_mask;
    c->tuned_nrhs = nrhs;
    tune_cache_store(c, sig);
}

// ---------------------------------------------------------------------------
// operator and preconditioner

// Workgroups of one operator application over the grid of (n1+1) x (n2+1)
// (x (n3+1)) points: tiles of OTX x OTY points (per plane in 3D).
inline dim3 op_grid(const eh_ctx* c) {
    Dims e = c->dcell;
    for (int a = 0; a < c->dim; ++a) e.g[a] += 1;
    return dim3((unsigned)((e.g[0] + OTX - 1) / OTX), (unsigned)((e.g[1] + OTY - 1) / OTY),
                (unsigned)(c->dim == 3 ? e.g[2] : 1));
}
inline int op_blocks(const eh_ctx* c) {
    const dim3 g = op_grid(c);
    return (int)(g.x * g.y * g.z);
}

template <class Tin, bool RES>
void launch_H(eh_ctx* c, const void* x, int64_t vx, c128* y, int64_t vy, int nrhs, ResArgs ra) {
    OpArgs o{};
    o.dc = c->dcell;
    for (int a = 0; a < 3; ++a) {
        o.ih[a] = 1.0 / c->h[a];
        if (a < c->dim) {
            o.df[a] = c->dface[a];
            for (int b = 0; b < 3; ++b) o.w[a][b] = c->k1w[a][b];
            o.D[a] = c->k1D[a];
        }
    }
    for (int a = 0; a < 4; ++a) o.off[a] = c->off[a];
    o.C = c->C;
    // a batch on a small grid is spread over chunks of right-hand sides in z
    const dim3 g = op_grid(c);
    const int rch = rhs_chunk((int)(g.x * g.y * g.z), 1, nrhs);
    const dim3 gc(g.x, g.y, g.z * (unsigned)((std::max(nrhs, 1) + rch - 1) / rch));
    if (c->dim == 2)
        hipLaunchKernelGGL((k_op2_lds<Tin, RES>), gc, dim3(256), 0, c->s, o, (const cplx<Tin>*)x, y, nrhs, vx, vy, ra,
                           rch);
    else
        hipLaunchKernelGGL((k_op3_lds<Tin, RES>), gc, dim3(256), 0, c->s, o, (const cplx<Tin>*)x, y, nrhs, vx, vy, ra,
                           rch);
    HIPCHK(hipGetLastError());
}

template <class Tin>
void apply_H(eh_ctx* c, const void* x, int64_t vx, c128* y, int64_t vy, int nrhs) {
    double coefb = 8.0 * c->ncell;
    for (int k = 0; k < c->dim; ++k) coefb += (double)c->fsize[k] * (8.0 * c->dim + 16.0);
    Timed tm(c, KC_OPERATOR, coefb + (double)nrhs * c->ndof * (sizeof(cplx<Tin>) + sizeof(c128)));
    launch_H<Tin, false>(c, x, vx, y, vy, nrhs, ResArgs{});
}

// w = H z for nrhs vectors in the multigrid precision and, from the same
// launch, the first Gram-Schmidt pass of the Arnoldi step: d1 row r =
// [conj(V_t) . w for t < J, conj(V_t) . V_{J-1} for t < J] with basis
// column t of RHS r at V + t * vstep + r * ndof.  2D only: in 3D the plane
// kernel with the pass folded in measured slower than the two launches
// (192^3 x 4: 486 against 461 ms per solve for operator and Krylov work),
// so there, and for more columns than the launch handles, it returns false
// (nothing launched).
template <class Tin>
bool apply_H_dots(eh_ctx* c, const void* z, c128* w, int nrhs, const c128* V, int64_t vstep, int J, c128* d1) {
    if (c->dim != 2 || J > OP_MAXJ) return false;
    double coefb = 8.0 * c->ncell;
    for (int k = 0; k < c->dim; ++k) coefb += (double)c->fsize[k] * (8.0 * c->dim + 16.0);
    Timed tm(c, KC_OPERATOR,
             coefb + (double)nrhs * c->ndof * (sizeof(cplx<Tin>) + sizeof(c128) + J * sizeof(c128)));
    OpArgs o{};
    o.dc = c->dcell;
    for (int a = 0; a < 3; ++a) {
        o.ih[a] = 1.0 / c->h[a];
        if (a < c->dim) {
            o.df[a] = c->dface[a];
            for (int b = 0; b < 3; ++b) o.w[a][b] = c->k1w[a][b];
            o.D[a] = c->k1D[a];
        }
    }
    for (int a = 0; a < 4; ++a) o.off[a] = c->off[a];
    o.C = c->C;
    const dim3 g = op_grid(c);
    const int rch = rhs_chunk((int)(g.x * g.y * g.z), 1, nrhs);
    const dim3 gc(g.x, g.y, g.z * (unsigned)((std::max(nrhs, 1) + rch - 1) / rch));
    DotArgs da{V, vstep, J, c->partial};
    hipLaunchKernelGGL((k_op2_lds<Tin, false, true>), gc, dim3(256), 0, c->s, o, (const cplx<Tin>*)z, w, nrhs,
                       c->ndof, c->ndof, ResArgs{}, rch, da);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_reduce_partials, dim3(2 * J, nrhs), dim3(256), 0, c->s, (int)(g.x * g.y * g.z), 2 * J,
                       nrhs, c->partial, d1);
    HIPCHK(hipGetLastError());
    return true;
}

// r = b - H x for nrhs complex128 vectors of stride ndof, and nrm[q] =
// |r_q|^2 (the cycle start of FGMRES) from the same launches.
void residual_H(eh_ctx* c, const c128* x, const c128* b, c128* r, int nrhs, c128* nrm) {
    const int nb = op_blocks(c);
    double coefb = 8.0 * c->ncell;
    for (int k = 0; k < c->dim; ++k) coefb += (double)c->fsize[k] * (8.0 * c->dim + 16.0);
    Timed tm(c, KC_OPERATOR, coefb + (double)nrhs * c->ndof * 3.0 * sizeof(c128));
    ResArgs ra{};
    ra.b = b;
    ra.partial = c->res_partial;
    ra.nblk = nb;
    ra.blk0 = 0;
    launch_H<double, true>(c, x, c->ndof, r, c->ndof, nrhs, ra);
    hipLaunchKernelGGL(k_reduce_partials, dim3(1, nrhs), dim3(256), 0, c->s, nb, 1, nrhs, c->res_partial, nrm);
    HIPCHK(hipGetLastError());
}

// z = P^{-1} D_L r: r complex128 (stride vr), z multigrid precision (stride vz)
//
// With rs given, the input of RHS q is rs[q * rss] times the stored r (an
// unnormalised Krylov column); the preconditioner is linear, so the scale
// is applied where r is read.
template <class T>
void apply_M(eh_ctx* c, const c128* r, int64_t vr, void* z, int64_t vz, int nrhs, const double* rs = nullptr,
             int64_t rss = 0) {
    ensure_mg_workspace(c, nrhs);
    const int d = c->dim;
    Block& Bp = c->blk[d];
    Level& Lp = Bp.lev[0];
    const c128* r2 = d == 3 ? r + c->off[2] : r;
    {
    Timed tm(c, KC_DISTRIBUTE, 24.0 * c->ncell + (double)nrhs * (c->ndof * 16.0 + c->ncell * sizeof(cplx<T>)));
    const dim3 g0 = grid_of(c->dcell);
    const int rch = rhs_chunk((int)(g0.x * g0.y * g0.z), 1, nrhs);
    const dim3 g(g0.x, g0.y, g0.z * (unsigned)((std::max(nrhs, 1) + rch - 1) / rch));
    auto launch = [&](auto tilde_tag) {
        constexpr bool TILDE = decltype(tilde_tag)::value;
        if (d == 2)
            hipLaunchKernelGGL((k_distribute<T, 2, TILDE>), g, kBlock, 0, c->s, c->dcell,
                               r + c->off[0], r + c->off[1], r2, r + c->off[d], c->mu, c->mcell,
                               c->omega * c->omega, 1.0 / c->h[0], 1.0 / c->h[1], 1.0 / c->h[2], (cplx<T>*)Lp.f,
                               nrhs, vr, c->ncell, rs, rss, rch);
        else
            hipLaunchKernelGGL((k_distribute<T, 3, TILDE>), g, kBlock, 0, c->s, c->dcell,
                               r + c->off[0], r + c->off[1], r2, r + c->off[d], c->mu, c->mcell,
                               c->omega * c->omega, 1.0 / c->h[0], 1.0 / c->h[1], 1.0 / c->h[2], (cplx<T>*)Lp.f,
                               nrhs, vr, c->ncell, rs, rss, rch);
    };
    if (c->o.ap_variant == 1) launch(std::true_type{});
    else launch(std::false_type{});
    HIPCHK(hipGetLastError());
    }
    cplx<T>* Z = (cplx<T>*)z;
    cplx<T>* ep = Z + c->off[d];
    {
        const int kinds[1] = {d};
        const void* f[1] = {Lp.f};
        const int64_t vf[1] = {c->ncell};
        void* out[1] = {ep};
        const int64_t vo[1] = {vz};
        gcycle<T>(c, kinds, 1, 0, f, vf, out, vo, false, nrhs);
    }
    int kinds[GMAX];
    const void* f[GMAX];
    int64_t vf[GMAX], vo[GMAX];
    void* out[GMAX];
    CoupleArgs ca{};
    ca.ns = d;
    ca.maxg2 = 1;
    ca.rs = rs;
    ca.rss = rss;
    double by = 0.0;
    for (int k = 0; k < d; ++k) {
        Level& Lk = c->blk[k].lev[0];
        kinds[k] = k;
        f[k] = Lk.f;
        vf[k] = Lk.d.np();
        out[k] = Z + c->off[k];
        vo[k] = vz;
        ca.kind[k] = k;
        ca.d[k] = Lk.d;
        ca.maxg2 = std::max(ca.maxg2, Lk.d.g[2]);
        ca.ru[k] = r + c->off[k];
        ca.g[k] = Lk.f;
        ca.vg[k] = Lk.d.np();
        ca.ih[k] = 1.0 / c->h[k];
        by += (double)nrhs * (Lk.d.np() * (16.0 + sizeof(cplx<T>)) + c->ncell * sizeof(cplx<T>));
    }
    {
        Timed tm(c, KC_COUPLE, by);
        int gx = 1, gy = 1;
        for (int k = 0; k < d; ++k) {
            gx = std::max(gx, (ca.d[k].g[0] + 63) / 64);
            gy = std::max(gy, (ca.d[k].g[1] + 3) / 4);
        }
        const int rch = rhs_chunk(gx * gy * ca.maxg2, d, nrhs);
        const int nch = (std::max(nrhs, 1) + rch - 1) / rch;
        hipLaunchKernelGGL((k_gcouple<T>), dim3(gx, gy, ca.maxg2 * d * nch), kBlock, 0, c->s, ca, c->dcell,
                           (const cplx<T>*)ep, nrhs, vr, vz, rch);
        HIPCHK(hipGetLastError());
    }
    gcycle<T>(c, kinds, d, 0, f, vf, out, vo, false, nrhs);
}

// ---------------------------------------------------------------------------
// Krylov helpers

void free_arn_status(eh_ctx* c) {
    if (c->arn_host) (void)hipHostFree(c->arn_host);
    c->arn_host = nullptr;
    c->arn_dev = nullptr;
}

void ensure_krylov(eh_ctx* c, int nrhs, int m) {
    if (nrhs <= c->kry_nrhs && m <= c->kry_m) return;
    HIPCHK(hipStreamSynchronize(c->s));
    drop_graphs(c);
    c->release(c->V); c->release(c->Z); c->release(c->W); c->release(c->partial); c->release(c->res_partial);
    c->release(c->dsmall);
    c->release(c->arn.sv);
    free_arn_status(c);
    c->V = c->alloc<c128>((size_t)(m + 1) * nrhs * c->ndof);
    c->Z = c->alloc<char>((size_t)m * nrhs * c->ndof * c->csize());
    c->W = c->alloc<c128>((size_t)nrhs * c->ndof);
    c->kry_nblk = (int)std::max<int64_t>(1, (c->ndof + KRY_E * KRY_THREADS - 1) / (KRY_E * KRY_THREADS));
    // Gram-Schmidt partials: the k_gs blocks, or the operator workgroups
    // where the 2D operator launch does the first pass
    c->partial = c->alloc<c128>((size_t)std::max(c->kry_nblk, op_blocks(c)) * nrhs * 2 * (m + 1));
    c->res_partial = c->alloc<c128>((size_t)op_blocks(c) * nrhs);
    c->dsmall = c->alloc<c128>((size_t)6 * nrhs * (m + 2));
    // Arnoldi state: one allocation carved into 16-byte aligned arrays
    const size_t R = nrhs, M = m;
    const size_t sizes[15] = {R * (M + 1) * sizeof(double), sizeof(double), R * M * M * sizeof(c128),
                              R * M * sizeof(c128), R * M * (M + 1) * sizeof(c128), R * M * sizeof(double),
                              R * M * sizeof(c128), R * (M + 1) * sizeof(c128), R * M * sizeof(c128),
                              R * sizeof(double), R * sizeof(double), R * sizeof(int), R * sizeof(int),
                              R * sizeof(int), R * sizeof(int)};
    size_t total16 = 0;
    for (size_t b : sizes) total16 += (b + 15) / 16;
    char* base = (char*)c->alloc<c128>(total16);
    int ti = 0;
    auto take = [&]() { char* p = base; base += (sizes[ti++] + 15) / 16 * 16; return p; };
    ArnState& A = c->arn;
    A.m = m;
    A.nrhs = nrhs;
    A.sv = (double*)take();     // first: the allocation's base (released through it)
    A.tol = (double*)take();
    A.gram = (c128*)take();
    A.hcol = (c128*)take();
    A.R = (c128*)take();
    A.cs = (double*)take();
    A.sn = (c128*)take();
    A.g = (c128*)take();
    A.y = (c128*)take();
    A.bnorm = (double*)take();
    A.est = (double*)take();
    A.jr = (int*)take();
    A.act = (int*)take();
    A.its = (int*)take();
    A.done = (int*)take();
    void* hp = nullptr;
    HIPCHK(hipHostMalloc(&hp, (M + 1) * R * sizeof(ArnStatus), hipHostMallocMapped | hipHostMallocCoherent));
    c->arn_host = (ArnStatus*)hp;
    void* dp = nullptr;
    HIPCHK(hipHostGetDevicePointer(&dp, hp, 0));
    c->arn_dev = (ArnStatus*)dp;
    std::memset(hp, 0, (M + 1) * R * sizeof(ArnStatus));
    while (c->arn_ev.size() < M + 1) {
        hipEvent_t e;
        HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        c->arn_ev.push_back(e);
    }
    c->kry_nrhs = nrhs;
    c->kry_m = m;
}

// Gram-Schmidt pass over columns [0, m): MODE as in k_gs.  coef/out are
// device arrays [nrhs][m] (out: [nrhs][1] for norms).
template <int MODE>
void gs_pass(eh_ctx* c, int64_t n, int m, int nrhs, const c128* V, const c128* w, const c128* coef, c128* out,
             c128* wout = nullptr) {
    const int nblk = (int)std::max<int64_t>(1, (n + KRY_E * KRY_THREADS - 1) / (KRY_E * KRY_THREADS));
    const double vecs = (MODE == 0 || MODE == 4) ? m + 1 : (MODE == 3 ? 1 : m + 2);
    Timed tm(c, KC_KRYLOV, vecs * nrhs * n * sizeof(c128));
    hipLaunchKernelGGL((k_gs<MODE>), dim3(nblk, nrhs), dim3(KRY_THREADS), 0, c->s, n, m, nrhs, V, w,
                       coef, c->partial, wout);
    HIPCHK(hipGetLastError());
    const int mm = (MODE == 0 || MODE == 1) ? m : (MODE == 4 ? 2 * m : 1);
    hipLaunchKernelGGL(k_reduce_partials, dim3(mm, nrhs), dim3(256), 0, c->s, nblk, mm, nrhs, c->partial, out);
    HIPCHK(hipGetLastError());
}

// Flexible GMRES(m) with right preconditioning, x_0 = 0.  Every Arnoldi
// step -- z_j = M v_j, w = H z_j, CGS2 against the basis and the Hessenberg
// update -- runs on the device (replayed from a HIP graph when enabled); the
// host reads the status record of step j-1 while step j runs and waits for
// step j itself only when the estimate is about to cross the tolerance, so
// at most one step is queued beyond convergence (it then acts on inactive
// right-hand sides only: scale 0, no column counted).  A cycle start
// computes r = b - H x in FP64, so the last start gives the true residual.
//
// The problem enters through four callbacks, each enqueueing on c->s for
// the nb right-hand sides currently in the batch:
//   op_x(x, W, nb)            W = X x for an FP64 vector (cycle starts)
//   op_z(z_j, W, nb)          W = X z_j for a preconditioned vector (multigrid precision)
//   op_zd(z_j, W, nb, V, vstep, J, d1)
//                             the same and the first Gram-Schmidt pass over
//                             columns 0..J-1 into d1 from the same launch, or
//                             false where the problem does not provide it
//   prec(v, sv, z_j, nb)      z_j = M (sv[q * (m+1)] v) per right-hand side q
//   op_res(x, b, r, nrm, nb)  r = b - X x and nrm = |r|^2 in one pass, or false
//                             where the problem does not provide it
// with vectors of length n, right-hand side q at offset q * n.  Graph
// capture is used only for the full system (`graphs`).
//
// With drop_converged, a cycle start whose true residuals show some right-
// hand sides finished (and some not) moves the unfinished ones to the first
// slots of the batch -- their x and b into buffers of this solve, their
// cycle-start residual within stored column 0, their Arnoldi state on the
// device -- and later launches cover only them.  A dropped right-hand side's
// x goes back to its place in the caller's x.  Every kernel's arithmetic per
// right-hand side does not depend on the batch around it, so the results
// and the counts are those of the full batch.
template <class T, class OpX, class OpZ, class OpZD, class Prec, class OpRes>
eh_status fgmres_core(eh_ctx* c, int64_t n, OpX op_x, OpZ op_z, OpZD op_zd, Prec prec, bool graphs, const c128* b,
                      c128* x, int nrhs, double tol, int maxit, eh_info* info, OpRes op_res) {
    const int m = c->o.restart;
    int nb = nrhs;                               // right-hand sides in the batch
    int64_t vstep = (int64_t)nb * n;             // distance between basis vectors
    cplx<T>* Z = (cplx<T>*)c->Z;
    ArnState S = c->arn;
    S.nrhs = nb;
    ArnStatus* hs = c->arn_host;
    ArnStatus* ds = c->arn_dev;
    c128* d1 = c->dsmall;
    c128* d2 = c->dsmall + (size_t)2 * nrhs * (m + 2);
    c128* d3 = c->dsmall + (size_t)4 * nrhs * (m + 2);
    unsigned rgrid = (unsigned)((nb + 63) / 64);
    // predicted estimate below this multiple of tol: wait for the step
    constexpr double kNear = 3.0;
    HIPCHK(hipMemsetAsync(x, 0, (size_t)nrhs * n * sizeof(c128), c->s));
    // the batch: slot q holds right-hand side orig[q] of the call; its b and
    // x live in the caller's arrays until the first drop, then in cbuf
    std::vector<int> orig(nrhs);
    for (int r = 0; r < nrhs; ++r) orig[r] = r;
    std::vector<ArnStatus> fin_all(nrhs);
    const c128* bw = b;
    c128* xw = x;
    struct Scratch {
        eh_ctx* c;
        c128* buf = nullptr;
        int* map = nullptr;
        ~Scratch() {
            if (buf || map) (void)hipStreamSynchronize(c->s);
            c->release(buf);
            c->release(map);
        }
    } scr{c};
    int total = 0;
    bool first = true;
    auto status = [&](int slot) { return hs + (size_t)slot * nrhs; };
    auto check_bad = [&](const ArnStatus* st) {
        for (int r = 0; r < nb; ++r)
            if (st[r].bad) throw StateError{"non-finite value in the Arnoldi process"};
    };
    auto any_active = [&](const ArnStatus* st) {
        for (int r = 0; r < nb; ++r)
            if (st[r].active) return true;
        return false;
    };
    auto copy_vec = [&](c128* dst, const c128* src) {
        HIPCHK(hipMemcpyAsync(dst, src, (size_t)n * sizeof(c128), hipMemcpyDeviceToDevice, c->s));
    };
    // Keep the slots listed in keep (increasing), drop the rest.  Called at a
    // cycle start, after k_arn_start and the host's read of its records.
    auto drop = [&](const std::vector<int>& keep) {
        const int k = (int)keep.size();
        ArnStatus* st = status(m);
        std::vector<char> kept(nb, 0);
        for (int q : keep) kept[q] = 1;
        for (int q = 0; q < nb; ++q)
            if (!kept[q]) fin_all[orig[q]] = st[q];
        if (xw == x) {
            // first drop: the dropped x are already in place; gather the rest
            scr.buf = c->alloc<c128>((size_t)2 * k * n);
            scr.map = c->alloc<int>((size_t)nrhs);
            c128* nx = scr.buf;
            c128* nbv = scr.buf + (size_t)k * n;
            for (int i = 0; i < k; ++i) {
                copy_vec(nx + (size_t)i * n, xw + (size_t)keep[i] * n);
                copy_vec(nbv + (size_t)i * n, bw + (size_t)keep[i] * n);
            }
            xw = nx;
            bw = nbv;
        } else {
            for (int q = 0; q < nb; ++q)
                if (!kept[q]) copy_vec(x + (size_t)orig[q] * n, xw + (size_t)q * n);
            for (int i = 0; i < k; ++i)
                if (keep[i] != i) {
                    copy_vec(xw + (size_t)i * n, xw + (size_t)keep[i] * n);
                    copy_vec((c128*)bw + (size_t)i * n, bw + (size_t)keep[i] * n);
                }
        }
        // stored column 0 holds the cycle-start residuals (slot q at q * n)
        for (int i = 0; i < k; ++i)
            if (keep[i] != i) copy_vec(c->V + (size_t)i * n, c->V + (size_t)keep[i] * n);
        HIPCHK(hipMemcpyAsync(scr.map, keep.data(), (size_t)k * sizeof(int), hipMemcpyHostToDevice, c->s));
        hipLaunchKernelGGL(k_arn_compact, dim3(1), dim3(64), 0, c->s, S, (const int*)scr.map, k);
        HIPCHK(hipGetLastError());
        // keep.data() must outlive the copy
        HIPCHK(hipStreamSynchronize(c->s));
        for (int i = 0; i < k; ++i) {
            st[i] = st[keep[i]];
            orig[i] = orig[keep[i]];
        }
        nb = k;
        S.nrhs = nb;
        vstep = (int64_t)nb * n;
        rgrid = (unsigned)((nb + 63) / 64);
    };
    for (;;) {
        // r = b - H x into stored column 0; its norm starts the cycle
        if (first) {
            HIPCHK(hipMemcpyAsync(c->V, bw, (size_t)vstep * sizeof(c128), hipMemcpyDeviceToDevice, c->s));
            gs_pass<3>(c, n, 1, nb, nullptr, c->V, nullptr, d3);
        } else if (!op_res(xw, bw, c->V, d3, nb)) {
            // (op_res: r and |r|^2 from the operator launch itself, where the
            // problem provides it)
            op_x(xw, c->W, nb);
            hipLaunchKernelGGL(k_sub, dim3(lin_grid(vstep, 256, 4096)), dim3(256), 0, c->s, vstep, bw, c->W, c->V);
            HIPCHK(hipGetLastError());
            gs_pass<3>(c, n, 1, nb, nullptr, c->V, nullptr, d3);
        }
        hipLaunchKernelGGL(k_arn_start, dim3(rgrid), dim3(64), 0, c->s, S, (const c128*)d3, first ? 1 : 0, tol,
                           ds + (size_t)m * nrhs);
        HIPCHK(hipGetLastError());
        first = false;
        HIPCHK(hipStreamSynchronize(c->s));
        check_bad(status(m));
        if (!any_active(status(m)) || total >= maxit) break;
        if (c->o.drop_converged) {
            std::vector<int> keep;
            for (int q = 0; q < nb; ++q)
                if (status(m)[q].active) keep.push_back(q);
            if ((int)keep.size() < nb) drop(keep);
        }
        int steps = 0;
        for (int j = 0; j < m && total < maxit; ++j) {
            c128* Vj = c->V + (int64_t)j * vstep;
            cplx<T>* Zj = Z + (int64_t)j * vstep;
            auto body = [&]() {
                prec(Vj, S.sv + j, Zj, nb);
                if (!op_zd(Zj, c->W, nb, c->V, vstep, j + 1, d1)) {
                    op_z(Zj, c->W, nb);
                    gs_pass<4>(c, n, j + 1, nb, c->V, c->W, nullptr, d1);
                }
                hipLaunchKernelGGL(k_arn_coef, dim3(nb), dim3(64), 0, c->s, S, j, (const c128*)d1, d2);
                HIPCHK(hipGetLastError());
                gs_pass<2>(c, n, j + 1, nb, c->V, c->W, d2, d3, Vj + vstep);
                hipLaunchKernelGGL(k_arn_givens, dim3(rgrid), dim3(64), 0, c->s, S, j, (const c128*)d3,
                                   ds + (size_t)j * nrhs);
                HIPCHK(hipGetLastError());
            };
            if (graphs && c->timer_mask == 0) {
                if (c->graph_nrhs != nb || c->graph_stride != nrhs || (int)c->graphs.size() != m) {
                    drop_graphs(c);
                    c->graphs.resize(m);
                    c->graph_nrhs = nb;
                    c->graph_stride = nrhs;
                }
                eh_ctx::GraphEntry& g = c->graphs[j];
                if (!g.exec) {
                    HIPCHK(hipStreamBeginCapture(c->s, hipStreamCaptureModeRelaxed));
                    c->capturing = true;
                    try {
                        body();
                    } catch (...) {
                        c->capturing = false;
                        hipGraph_t tmp = nullptr;
                        (void)hipStreamEndCapture(c->s, &tmp);
                        if (tmp) (void)hipGraphDestroy(tmp);
                        throw;
                    }
                    c->capturing = false;
                    HIPCHK(hipStreamEndCapture(c->s, &g.graph));
                    HIPCHK(hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0));
                }
                HIPCHK(hipGraphLaunch(g.exec, c->s));
            } else {
                body();
            }
            HIPCHK(hipEventRecord(c->arn_ev[j], c->s));
            ++total;
            ++steps;
            if (j == m - 1 || total >= maxit) break;
            // Is step j+1 needed?  Known: the status after step j-1 (the
            // cycle start for j = 0); step j is still running.
            const ArnStatus* known = status(j == 0 ? m : j - 1);
            if (j > 0) HIPCHK(hipEventSynchronize(c->arn_ev[j - 1]));
            check_bad(known);
            if (!any_active(known)) break;
            const ArnStatus* before = j >= 2 ? status(j - 2) : (j == 1 ? status(m) : nullptr);
            bool near = true;
            for (int r = 0; r < nb && near; ++r) {
                if (!known[r].active) continue;
                double ratio = 1.0;
                if (before && before[r].est > 0.0) ratio = std::min(1.0, known[r].est / before[r].est);
                if (known[r].est * ratio >= kNear * tol) near = false;
            }
            if (near) {
                HIPCHK(hipEventSynchronize(c->arn_ev[j]));
                check_bad(status(j));
                if (!any_active(status(j))) break;
            }
        }
        // x += Z y with y = R^-1 g of this cycle
        hipLaunchKernelGGL(k_arn_solve, dim3(rgrid), dim3(64), 0, c->s, S);
        HIPCHK(hipGetLastError());
        {
            Timed tm(c, KC_KRYLOV, (double)nb * n * (2 * sizeof(c128) + steps * sizeof(cplx<T>)));
            hipLaunchKernelGGL((k_xupdate<T>), dim3(lin_grid(n, 256, 2048), nb), dim3(256), 0, c->s, n,
                               (const int*)S.jr, m, nb, (const cplx<T>*)Z, (const c128*)S.y, xw);
            HIPCHK(hipGetLastError());
        }
    }
    // the last cycle start computed the true FP64 residual of x
    const ArnStatus* fin = status(m);
    for (int q = 0; q < nb; ++q) {
        fin_all[orig[q]] = fin[q];
        if (xw != x) copy_vec(x + (size_t)orig[q] * n, xw + (size_t)q * n);
    }
    bool all = true;
    for (int r = 0; r < nrhs; ++r) {
        const int conv = fin_all[r].rel < tol;
        all = all && conv;
        if (info) {
            info[r].iters = fin_all[r].its;
            info[r].converged = conv;
            info[r].relres_true = fin_all[r].rel;
            info[r].relres_est = fin_all[r].est;
        }
    }
    return all ? EH_OK : EH_NOT_CONVERGED;
}

// The full system: H x = b with the block-acoustic preconditioner.
template <class T>
eh_status solve_impl(eh_ctx* c, const c128* b, c128* x, int nrhs, double tol, int maxit, eh_info* info) {
    ensure_krylov(c, nrhs, c->o.restart);
    ensure_mg_workspace(c, nrhs);     // no allocation may happen inside a graph capture
    maybe_autotune<T>(c, nrhs);
    const int64_t n = c->ndof;
    const int m = c->o.restart;
    auto op_x = [&](const c128* xx, c128* w, int nb) { apply_H<double>(c, xx, n, w, n, nb); };
    auto op_z = [&](const cplx<T>* z, c128* w, int nb) { apply_H<T>(c, z, n, w, n, nb); };
    auto op_res = [&](const c128* xx, const c128* bb, c128* r, c128* nrm, int nb) {
        residual_H(c, xx, bb, r, nb, nrm);
        return true;
    };
    auto prec = [&](const c128* v, const double* sv, cplx<T>* z, int nb) {
        apply_M<T>(c, v, n, z, n, nb, sv, m + 1);
    };
    auto op_zd = [&](const cplx<T>* z, c128* w, int nb, const c128* V, int64_t vstep, int J, c128* d1) {
        return apply_H_dots<T>(c, z, w, nb, V, vstep, J, d1);
    };
    return fgmres_core<T>(c, n, op_x, op_z, op_zd, prec, c->o.graphs != 0, b, x, nrhs, tol, maxit, info, op_res);
}

eh_status fail(eh_ctx* c, eh_status st, const std::string& msg);

// One acoustic block alone: X_b x = f on the fine grid with FGMRES, right-
// preconditioned by the block's multigrid cycle (the shifted operator of
// the block, as inverted inside the preconditioner).  The operator is
// applied in the multigrid precision.
template <class T>
eh_status block_solve_impl(eh_ctx* c, int block, const c128* f, c128* x, int nrhs, double tol, int maxit,
                           eh_info* info) {
    ensure_krylov(c, nrhs, c->o.restart);
    ensure_mg_workspace(c, nrhs);
    maybe_autotune<T>(c, nrhs);
    Level& L = c->blk[block].lev[0];
    const int64_t n = L.d.np();
    const int m = c->o.restart;
    const int kinds[1] = {block};
    auto apply_T = [&](const cplx<T>* u, int64_t vu, c128* w, int nb) {
        GArgs<T> a = gbase<T>(c, kinds, 1, 0, false);
        a.u[0] = u;
        a.vu[0] = vu;
        a.out[0] = (cplx<T>*)L.t;
        a.vo[0] = n;
        gsweep<T>(c, a, 0, 3, nb);
        hipLaunchKernelGGL((k_cast<double, T>), dim3(lin_grid(n * nb, 256, 8192)), dim3(256), 0, c->s,
                           n * nb, (const cplx<T>*)L.t, w);
        HIPCHK(hipGetLastError());
    };
    auto op_x = [&](const c128* xx, c128* w, int nb) {
        hipLaunchKernelGGL((k_cast_scaled<T>), dim3(lin_grid(n, 256, 4096), nb), dim3(256), 0, c->s, n, xx, n,
                           (const double*)nullptr, (int64_t)0, (cplx<T>*)L.u, n);
        HIPCHK(hipGetLastError());
        apply_T((const cplx<T>*)L.u, n, w, nb);
    };
    auto op_z = [&](const cplx<T>* z, c128* w, int nb) { apply_T(z, n, w, nb); };
    auto prec = [&](const c128* v, const double* sv, cplx<T>* z, int nb) {
        hipLaunchKernelGGL((k_cast_scaled<T>), dim3(lin_grid(n, 256, 4096), nb), dim3(256), 0, c->s, n, v, n,
                           sv, (int64_t)(m + 1), (cplx<T>*)L.f, n);
        HIPCHK(hipGetLastError());
        const void* fa[1] = {L.f};
        const int64_t vf[1] = {n};
        void* out[1] = {z};
        gcycle<T>(c, kinds, 1, 0, fa, vf, out, vf, false, nb);
    };
    auto no_res = [](const c128*, const c128*, c128*, c128*, int) { return false; };
    auto no_zd = [](const cplx<T>*, c128*, int, const c128*, int64_t, int, c128*) { return false; };
    return fgmres_core<T>(c, n, op_x, op_z, no_zd, prec, false, f, x, nrhs, tol, maxit, info, no_res);
}

void ensure_zbuf(eh_ctx* c) {
    if (c->zbuf) return;
    c->zbuf = c->alloc<c128>((size_t)2 * c->ndof);
    c->zy = c->alloc<c128>((size_t)c->ncell);
}

// y = Z(alpha) v = Xi A_alpha^-1 B^T H_p,alpha^-1 v for one cell vector
// (eq. Z with the preconditioner's shifted blocks; Xi = B A - A_p B, or
// B A - A~_p B with the Remark's variant).  The inverses are block solves
// to `tol`; with w = A_alpha^-1 B^T t, Xi w is the distributor applied to
// H [w; 0] = [A w; B w].
template <class T>
eh_status apply_Z_impl(eh_ctx* c, const c128* v, c128* y, double tol, int maxit) {
    ensure_zbuf(c);
    const int d = c->dim;
    c128* z1 = c->zbuf;
    c128* z2 = c->zbuf + c->ndof;
    eh_info inf{};
    hipLaunchKernelGGL((k_fill<c128>), dim3(lin_grid(c->ndof, 256, 4096)), dim3(256), 0, c->s, c->ndof, z1,
                       mk(0.0, 0.0));
    HIPCHK(hipGetLastError());
    eh_status st = block_solve_impl<T>(c, d, v, z1 + c->off[d], 1, tol, maxit, &inf);
    if (st != EH_OK) return st == EH_NOT_CONVERGED ? fail(c, st, "inner H_p solve did not converge") : st;
    apply_H<double>(c, z1, c->ndof, z2, c->ndof, 1);            // u rows: B^T t
    for (int k = 0; k < d; ++k) {
        st = block_solve_impl<T>(c, k, z2 + c->off[k], z1 + c->off[k], 1, tol, maxit, &inf);
        if (st != EH_OK) return st == EH_NOT_CONVERGED ? fail(c, st, "inner A_k solve did not converge") : st;
    }
    hipLaunchKernelGGL((k_fill<c128>), dim3(lin_grid(c->ncell, 256, 4096)), dim3(256), 0, c->s, c->ncell,
                       z1 + c->off[d], mk(0.0, 0.0));
    HIPCHK(hipGetLastError());
    apply_H<double>(c, z1, c->ndof, z2, c->ndof, 1);            // [A w; B w]
    const c128* r2 = d == 3 ? z2 + c->off[2] : z2;
    auto launch = [&](auto tilde_tag) {
        constexpr bool TILDE = decltype(tilde_tag)::value;
        if (d == 2)
            hipLaunchKernelGGL((k_distribute<double, 2, TILDE>), grid_of(c->dcell), kBlock, 0, c->s, c->dcell,
                               z2 + c->off[0], z2 + c->off[1], r2, z2 + c->off[d], c->mu, c->mcell,
                               c->omega * c->omega, 1.0 / c->h[0], 1.0 / c->h[1], 1.0 / c->h[2], y, 1, c->ndof,
                               c->ncell, (const double*)nullptr, (int64_t)0, 1);
        else
            hipLaunchKernelGGL((k_distribute<double, 3, TILDE>), grid_of(c->dcell), kBlock, 0, c->s, c->dcell,
                               z2 + c->off[0], z2 + c->off[1], r2, z2 + c->off[d], c->mu, c->mcell,
                               c->omega * c->omega, 1.0 / c->h[0], 1.0 / c->h[1], 1.0 / c->h[2], y, 1, c->ndof,
                               c->ncell, (const double*)nullptr, (int64_t)0, 1);
    };
    if (c->o.ap_variant == 1) launch(std::true_type{});
    else launch(std::false_type{});
    HIPCHK(hipGetLastError());
    return EH_OK;
}

// ||w||_2 of one vector of length n (deterministic reduction), synchronising
double norm2(eh_ctx* c, const c128* w, int64_t n) {
    c128* d = c->dsmall;
    gs_pass<3>(c, n, 1, 1, nullptr, w, nullptr, d);
    c128 h;
    HIPCHK(hipMemcpyAsync(&h, d, sizeof(c128), hipMemcpyDeviceToHost, c->s));
    HIPCHK(hipStreamSynchronize(c->s));
    return std::sqrt(std::max(0.0, h.re));
}

// Power method on Z(alpha) (Section 5: rho(Z) as a function of the shift):
// v <- Z v / ||Z v|| from the caller's v (normalised first), est[k] =
// ||Z v_k||.  v holds the last iterate on return.
template <class T>
eh_status power_Z_impl(eh_ctx* c, c128* v, int iters, double tol, int maxit, double* est) {
    ensure_krylov(c, 1, c->o.restart);
    ensure_zbuf(c);
    const int64_t nc = c->ncell;
    const double nv = norm2(c, v, nc);
    if (!(nv > 0.0) || !std::isfinite(nv)) return fail(c, EH_ERR_ARG, "power method start vector is zero or not finite");
    hipLaunchKernelGGL(k_scal, dim3(lin_grid(nc, 256, 4096)), dim3(256), 0, c->s, nc, 1.0 / nv, v, v);
    HIPCHK(hipGetLastError());
    for (int k = 0; k < iters; ++k) {
        eh_status st = apply_Z_impl<T>(c, v, c->zy, tol, maxit);
        if (st != EH_OK) return st;
        const double ny = norm2(c, c->zy, nc);
        est[k] = ny;
        if (!std::isfinite(ny)) return fail(c, EH_ERR_STATE, "non-finite value in the power method");
        if (ny == 0.0) {
            for (int q = k + 1; q < iters; ++q) est[q] = 0.0;
            break;
        }
        hipLaunchKernelGGL(k_scal, dim3(lin_grid(nc, 256, 4096)), dim3(256), 0, c->s, nc, 1.0 / ny,
                           (const c128*)c->zy, v);
        HIPCHK(hipGetLastError());
    }
    HIPCHK(hipStreamSynchronize(c->s));
    return EH_OK;
}

eh_status fail(eh_ctx* c, eh_status st, const std::string& msg) {
    if (c) c->err = msg;
    return st;
}

eh_status from_hip(eh_ctx* c, const HipError& e) {
    std::string m = std::string("HIP error ") + hipGetErrorString(e.e) + " in " + e.where;
    if (c) { c->err = m; c->broken = true; }
    else g_create_error = m;
    return e.e == hipErrorOutOfMemory ? EH_ERR_OOM : EH_ERR_HIP;
}

void destroy_all(eh_ctx* c) {
    drop_graphs(c);
    free_arn_status(c);
    for (auto e : c->arn_ev) (void)hipEventDestroy(e);
    c->arn_ev.clear();
    if (c->solve_stream) { (void)hipStreamDestroy(c->solve_stream); c->solve_stream = nullptr; }
    if (c->order_event) { (void)hipEventDestroy(c->order_event); c->order_event = nullptr; }
    for (auto& r : c->timer_recs) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
    c->timer_recs.clear();
    for (auto e : c->event_pool) (void)hipEventDestroy(e);
    c->event_pool.clear();
    for (void* p : c->allocs) (void)hipFree(p);
    c->allocs.clear();
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

void eh_default_opts(eh_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->levels = 3;
    o->cycle = 0;
    o->nu_pre = 1;
    o->nu_post = 2;
    o->n_damping = 3;
    o->damping[0] = 0.8;
    o->damping[1] = 0.8;
    o->damping[2] = 0.3;
    o->alpha = 0.1;
    o->mg_precision = 32;
    o->restart = 20;
    o->abc_width = 20;
    o->abc_sides = 0;   // filled per dim in eh_create when zero: all but the top
    o->gamma0 = 0.01 * M_PI;
    o->intergrid = 0;
    o->graphs = 1;
    o->autotune = 1;
    o->fused = 1;
    o->ap_variant = 0;
    o->coarse_solver = 0;
    o->drop_converged = 1;
}

const char* eh_last_error(const eh_ctx* c) {
    if (!c) return g_create_error.c_str();
    return c->err.c_str();
}

int64_t eh_ndof(const eh_ctx* c) { return c ? c->ndof : 0; }

eh_status eh_create(eh_ctx** out, int dim, const int64_t* n, const double* h, const double* vp,
                    const double* vs, const double* rho, double omega, const eh_opts* opts, void* stream) {
    g_create_error.clear();
    if (!out) { g_create_error = "ctx pointer is NULL"; return EH_ERR_ARG; }
    *out = nullptr;
    if (dim != 2 && dim != 3) { g_create_error = "dim must be 2 or 3"; return EH_ERR_ARG; }
    if (!n || !h || !vp || !vs || !rho) { g_create_error = "NULL array argument"; return EH_ERR_ARG; }
    if (!(omega > 0.0) || !std::isfinite(omega)) { g_create_error = "omega must be positive"; return EH_ERR_ARG; }
    eh_opts o;
    if (opts) o = *opts; else eh_default_opts(&o);
    if (o.abc_sides == 0 && !opts) {
        o.abc_sides = (1u << (2 * dim)) - 1u;
        o.abc_sides &= ~(1u << (2 * (dim - 1)));
    }
    if (o.levels < 1 || o.levels > 12) { g_create_error = "levels must be in [1, 12]"; return EH_ERR_ARG; }
    if (o.cycle != 0 && o.cycle != 1) { g_create_error = "cycle must be 0 (V) or 1 (W)"; return EH_ERR_ARG; }
    if (o.nu_pre < 0 || o.nu_post < 0 || o.nu_pre + o.nu_post < 1 || o.nu_pre > 16 || o.nu_post > 16) {
        g_create_error = "invalid smoothing counts"; return EH_ERR_ARG;
    }
    if (o.n_damping < 1 || o.n_damping > 8) { g_create_error = "n_damping must be in [1, 8]"; return EH_ERR_ARG; }
    if (o.mg_precision != 32 && o.mg_precision != 64) { g_create_error = "mg_precision must be 32 or 64"; return EH_ERR_ARG; }
    if (o.restart < 1 || o.restart > KRY_MAXM) { g_create_error = "restart must be in [1, 32]"; return EH_ERR_ARG; }
    if (o.abc_width < 0) { g_create_error = "abc_width must be >= 0"; return EH_ERR_ARG; }
    if (o.intergrid != 0 && o.intergrid != 1) { g_create_error = "intergrid must be 0 (full) or 1 (mixed)"; return EH_ERR_ARG; }
    if (o.graphs != 0 && o.graphs != 1) { g_create_error = "graphs must be 0 or 1"; return EH_ERR_ARG; }
    if (o.autotune != 0 && o.autotune != 1) { g_create_error = "autotune must be 0 or 1"; return EH_ERR_ARG; }
    if (o.fused != 0 && o.fused != 1) { g_create_error = "fused must be 0 or 1"; return EH_ERR_ARG; }
    if (o.drop_converged != 0 && o.drop_converged != 1) {
        g_create_error = "drop_converged must be 0 or 1"; return EH_ERR_ARG;
    }
    if (o.ap_variant != 0 && o.ap_variant != 1) { g_create_error = "ap_variant must be 0 or 1"; return EH_ERR_ARG; }
    if (o.coarse_solver < 0 || o.coarse_solver > 2) {
        g_create_error = "coarse_solver must be 0 (auto), 1 (dense) or 2 (block-tridiagonal)"; return EH_ERR_ARG;
    }
    if (!(o.alpha >= 0.0) || !std::isfinite(o.alpha)) { g_create_error = "alpha must be >= 0"; return EH_ERR_ARG; }
    int64_t ncell = 1;
    for (int a = 0; a < dim; ++a) {
        if (n[a] < 2 || n[a] > (1 << 20)) { g_create_error = "grid size out of range"; return EH_ERR_ARG; }
        if (n[a] % (int64_t(1) << (o.levels - 1)) != 0) {
            g_create_error = "each n must be divisible by 2^(levels-1)"; return EH_ERR_ARG;
        }
        if (!(h[a] > 0.0) || !std::isfinite(h[a])) { g_create_error = "h must be positive"; return EH_ERR_ARG; }
        ncell *= n[a];
    }
    if (dim == 2 && n[1] > 65535 * 4) { g_create_error = "grid too tall"; return EH_ERR_ARG; }
    for (int64_t q = 0; q < ncell; ++q) {
        if (!(rho[q] > 0.0) || !(vs[q] > 0.0) || !(vp[q] > vs[q]) || !std::isfinite(vp[q]) ||
            !std::isfinite(rho[q])) {
            g_create_error = "medium must satisfy vp > vs > 0 and rho > 0 (finite) in every cell";
            return EH_ERR_ARG;
        }
    }
    // coarsest solver: the dense inverse while every block's coarsest grid
    // has at most kDenseMax points (auto), else block-tridiagonal
    int64_t nc_max = 0;
    for (int b = 0; b <= dim; ++b) {
        int64_t np = 1;
        for (int a = 0; a < dim; ++a) np *= (n[a] >> (o.levels - 1)) + (b == a ? 1 : 0);
        nc_max = std::max(nc_max, np);
    }
    if (o.coarse_solver == 1 && nc_max > kDenseMax) {
        g_create_error = "coarsest grid too large for the dense direct solve (use coarse_solver 0 or 2)";
        return EH_ERR_ARG;
    }
    eh_ctx* c = new (std::nothrow) eh_ctx();
    if (!c) { g_create_error = "out of host memory"; return EH_ERR_OOM; }
    c->use_bt = o.coarse_solver == 2 || (o.coarse_solver == 0 && nc_max > kDenseMax);
    try {
        c->dim = dim;
        for (int a = 0; a < 3; ++a) { c->n[a] = a < dim ? n[a] : 1; c->h[a] = a < dim ? h[a] : 1.0; }
        c->omega = omega;
        c->o = o;
        c->s = (hipStream_t)stream;
        HIPCHK(hipGetDevice(&c->device));
        if (!setup_misfit_scratch(c->device)) throw HipError{hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)"};
        c->dcell = Dims{{(int)c->n[0], (int)c->n[1], (int)c->n[2]}};
        c->ncell = ncell;
        int64_t acc = 0;
        for (int k = 0; k < dim; ++k) {
            Dims d = c->dcell;
            d.g[k] += 1;
            c->dface[k] = d;
            c->off[k] = acc;
            c->fsize[k] = d.np();
            acc += d.np();
        }
        c->off[dim] = acc;
        c->fsize[dim] = ncell;
        c->ndof = acc + ncell;
        c->nblocks = dim + 1;
        // medium
        HostMedium M;
        M.mu.resize(ncell); M.lm.resize(ncell); M.rho.resize(ncell); M.gamma.resize(ncell); M.m.resize(ncell);
        for (int z = 0; z < c->n[2]; ++z)
            for (int y = 0; y < c->n[1]; ++y)
                for (int x = 0; x < c->n[0]; ++x) {
                    const int64_t q = cidx(c, x, y, z);
                    M.mu[q] = rho[q] * vs[q] * vs[q];
                    M.lm[q] = rho[q] * (vp[q] * vp[q] - vs[q] * vs[q]);
                    M.rho[q] = rho[q];
                    M.gamma[q] = abc_gamma(c, x, y, z);
                    M.m[q] = rho[q] * std::complex<double>(1.0, -M.gamma[q] / omega);
                }
        // FP64 arrays for H, the distributor and the gradient
        {
            std::vector<double> Cv(ncell);
            for (int64_t q = 0; q < ncell; ++q) Cv[q] = 1.0 / M.lm[q];
            upload_real<double>(c, (void**)&c->C, Cv);
            upload_real<double>(c, (void**)&c->mu, M.mu);
            upload_cplx<double>(c, (void**)&c->mcell, M.m);
            upload_real<double>(c, (void**)&c->d_rho, M.rho);
            upload_real<double>(c, (void**)&c->d_gamma, M.gamma);
            upload_real<double>(c, (void**)&c->d_lm, M.lm);
            std::vector<double> tmp(vp, vp + ncell);
            upload_real<double>(c, (void**)&c->d_vp, tmp);
            tmp.assign(vs, vs + ncell);
            upload_real<double>(c, (void**)&c->d_vs, tmp);
        }
        const bool f32 = o.mg_precision == 32;
        for (int b = 0; b <= dim; ++b) {
            Block& B = c->blk[b];
            B.kind = b;
            B.nodal_mask = b < dim ? (1 << b) : 0;
            B.lev.resize(o.levels);
            for (int l = 0; l < o.levels; ++l) {
                Dims d{};
                for (int a = 0; a < 3; ++a) {
                    const int64_t na = a < dim ? (c->n[a] >> l) : 1;
                    d.g[a] = (int)(na + ((B.nodal_mask >> a) & 1));
                }
                B.lev[l].d = d;
                B.lev[l].damp = o.damping[std::min(l, o.n_damping - 1)];
            }
            std::vector<double> w[3];
            std::vector<std::complex<double>> D, D0;
            if (b < dim) {
                build_Ak(c, M, b, o.alpha, w, D);
                std::vector<double> w0[3];
                build_Ak(c, M, b, 0.0, w0, D0);
                for (int a = 0; a < dim; ++a) upload_real<double>(c, (void**)&c->k1w[b][a], w0[a]);
                upload_cplx<double>(c, (void**)&c->k1D[b], D0);
                for (int a = 0; a < dim; ++a) {
                    if (f32) upload_real<float>(c, &B.fw[a], w[a]);
                    else upload_real<double>(c, &B.fw[a], w[a]);
                }
            } else if (o.ap_variant == 1) {
                build_Hp_tilde(c, M, o.alpha, w, D);
                for (int a = 0; a < dim; ++a) {
                    if (f32) upload_real<float>(c, &B.fw[a], w[a]);
                    else upload_real<double>(c, &B.fw[a], w[a]);
                }
            } else {
                build_Hp(c, M, o.alpha, w[0], D);
                if (f32) upload_real<float>(c, &B.fw[0], w[0]);
                else upload_real<double>(c, &B.fw[0], w[0]);
            }
            if (f32) upload_cplx<float>(c, &B.fD, D);
            else upload_cplx<double>(c, &B.fD, D);
            const std::vector<c128> st0 = fine_stencil(c, B, w, D);
            build_hierarchy(c, B, st0);
        }
        ensure_mg_workspace(c, 1);
        HIPCHK(hipDeviceSynchronize());
    } catch (const HipError& e) {
        from_hip(nullptr, e);
        destroy_all(c);
        delete c;
        return e.e == hipErrorOutOfMemory ? EH_ERR_OOM : EH_ERR_HIP;
    } catch (const ArgError& e) {
        g_create_error = e.msg;
        destroy_all(c);
        delete c;
        return EH_ERR_ARG;
    } catch (const std::bad_alloc&) {
        g_create_error = "out of host memory";
        destroy_all(c);
        delete c;
        return EH_ERR_OOM;
    }
    *out = c;
    return EH_OK;
}

void eh_destroy(eh_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->s);
    destroy_all(c);
    delete c;
}

eh_status eh_timer_enable(eh_ctx* c, unsigned class_mask) {
    if (!c || class_mask >= (1u << KC_COUNT)) return EH_ERR_ARG;
    c->timer_mask = class_mask;
    return EH_OK;
}

eh_status eh_timer_read(eh_ctx* c, int cls, int64_t* launches, double* ms, double* bytes) {
    if (!c || cls < 0 || cls >= KC_COUNT || !launches || !ms || !bytes) return EH_ERR_ARG;
    try {
        int64_t cnt = 0;
        double t = 0.0, by = 0.0;
        std::vector<eh_ctx::TimerRec> keep;
        for (auto& r : c->timer_recs) {
            if (r.cls != cls) { keep.push_back(r); continue; }
            HIPCHK(hipEventSynchronize(r.b));
            float e = 0.f;
            HIPCHK(hipEventElapsedTime(&e, r.a, r.b));
            t += e;
            by += r.bytes;
            ++cnt;
            c->event_pool.push_back(r.a);
            c->event_pool.push_back(r.b);
        }
        c->timer_recs.swap(keep);
        *launches = cnt;
        *ms = t;
        *bytes = by;
    } catch (const HipError& e) { return from_hip(c, e); }
    return EH_OK;
}

eh_status eh_set_stream(eh_ctx* c, void* stream) {
    if (!c) return EH_ERR_ARG;
    c->s = (hipStream_t)stream;
    return EH_OK;
}

#define EH_GUARD(c)                                             \
    if (!(c)) return EH_ERR_ARG;                                \
    if ((c)->broken) return fail((c), EH_ERR_STATE, "context unusable after an earlier HIP error");

eh_status eh_apply_operator(eh_ctx* c, const void* x, void* y, int nrhs) {
    EH_GUARD(c)
    if (!x || !y || nrhs < 1) return fail(c, EH_ERR_ARG, "invalid buffers or nrhs");
    try {
        apply_H<double>(c, x, c->ndof, (c128*)y, c->ndof, nrhs);
    } catch (const HipError& e) { return from_hip(c, e); }
    return EH_OK;
}

eh_status eh_apply_preconditioner(eh_ctx* c, const void* r, void* z, int nrhs) {
    EH_GUARD(c)
    if (!r || !z || nrhs < 1) return fail(c, EH_ERR_ARG, "invalid buffers or nrhs");
    try {
        if (c->o.mg_precision == 64) {
            maybe_autotune<double>(c, nrhs);
            apply_M<double>(c, (const c128*)r, c->ndof, z, c->ndof, nrhs);
        } else {
            ensure_tmpT(c, (int64_t)nrhs * c->ndof);
            maybe_autotune<float>(c, nrhs);
            apply_M<float>(c, (const c128*)r, c->ndof, c->tmpT, c->ndof, nrhs);
            const int64_t tot = (int64_t)nrhs * c->ndof;
            hipLaunchKernelGGL((k_cast<double, float>), dim3(lin_grid(tot, 256, 8192)), dim3(256), 0, c->s, tot,
                               (const c64*)c->tmpT, (c128*)z);
            HIPCHK(hipGetLastError());
        }
    } catch (const HipError& e) { return from_hip(c, e); }
    return EH_OK;
}

eh_status eh_block_dims(const eh_ctx* c, int block, int level, int64_t* out) {
    if (!c || !out || block < 0 || block > c->dim || level < 0 || level >= c->o.levels) return EH_ERR_ARG;
    for (int a = 0; a < 3; ++a) out[a] = c->blk[block].lev[level].d.g[a];
    return EH_OK;
}

}  // extern "C"

namespace {
template <class T>
void block_cycle_T(eh_ctx* c, int block, const void* f, void* e, int nrhs) {
    ensure_mg_workspace(c, nrhs);
    Block& B = c->blk[block];
    Level& L = B.lev[0];
    const int64_t np = L.d.np();
    const int64_t tot = np * nrhs;
    hipLaunchKernelGGL((k_cast<T, double>), dim3(lin_grid(tot, 256, 8192)), dim3(256), 0, c->s, tot,
                       (const c128*)f, (cplx<T>*)L.f);
    HIPCHK(hipGetLastError());
    ensure_tmpT(c, tot);
    const int kinds[1] = {block};
    const void* fa[1] = {L.f};
    const int64_t vf[1] = {np};
    void* out[1] = {c->tmpT};
    gcycle<T>(c, kinds, 1, 0, fa, vf, out, vf, false, nrhs);
    hipLaunchKernelGGL((k_cast<double, T>), dim3(lin_grid(tot, 256, 8192)), dim3(256), 0, c->s, tot,
                       (const cplx<T>*)c->tmpT, (c128*)e);
    HIPCHK(hipGetLastError());
}

template <class T>
void block_apply_T(eh_ctx* c, int block, int level, const void* x, void* y, int nrhs) {
    ensure_mg_workspace(c, nrhs);
    Block& B = c->blk[block];
    Level& L = B.lev[level];
    const int64_t np = L.d.np();
    const int64_t tot = np * nrhs;
    hipLaunchKernelGGL((k_cast<T, double>), dim3(lin_grid(tot, 256, 8192)), dim3(256), 0, c->s, tot,
                       (const c128*)x, (cplx<T>*)L.u);
    HIPCHK(hipGetLastError());
    const int kinds[1] = {block};
    GArgs<T> a = gbase<T>(c, kinds, 1, level, false);
    a.u[0] = (const cplx<T>*)L.u;
    a.vu[0] = np;
    a.out[0] = (cplx<T>*)L.t;
    a.vo[0] = np;
    gsweep<T>(c, a, level, 3, nrhs);
    hipLaunchKernelGGL((k_cast<double, T>), dim3(lin_grid(tot, 256, 8192)), dim3(256), 0, c->s, tot,
                       (const cplx<T>*)L.t, (c128*)y);
    HIPCHK(hipGetLastError());
}
}  // namespace

extern "C" {

eh_status eh_block_cycle(eh_ctx* c, int block, const void* f, void* e, int nrhs) {
    EH_GUARD(c)
    if (block < 0 || block > c->dim || !f || !e || nrhs < 1) return fail(c, EH_ERR_ARG, "invalid block or buffers");
    try {
        if (c->o.mg_precision == 64) block_cycle_T<double>(c, block, f, e, nrhs);
        else block_cycle_T<float>(c, block, f, e, nrhs);
    } catch (const HipError& er) { return from_hip(c, er); }
    return EH_OK;
}

eh_status eh_block_apply(eh_ctx* c, int block, int level, const void* x, void* y, int nrhs) {
    EH_GUARD(c)
    if (block < 0 || block > c->dim || level < 0 || level >= c->o.levels || !x || !y || nrhs < 1)
        return fail(c, EH_ERR_ARG, "invalid block, level or buffers");
    try {
        if (c->o.mg_precision == 64) block_apply_T<double>(c, block, level, x, y, nrhs);
        else block_apply_T<float>(c, block, level, x, y, nrhs);
    } catch (const HipError& er) { return from_hip(c, er); }
    return EH_OK;
}

eh_status eh_solve(eh_ctx* c, const void* b, void* x, int nrhs, double tol, int maxit, eh_info* info) {
    EH_GUARD(c)
    if (!b || !x || nrhs < 1 || !(tol > 0.0) || maxit < 0) return fail(c, EH_ERR_ARG, "invalid solve arguments");
    hipStream_t user = c->s;
    try {
        // the solve runs on the context's own stream (graphs cannot be
        // captured on the legacy default stream), ordered after the user's
        // stream by an event; the host waits for it before returning
        if (!c->solve_stream) HIPCHK(hipStreamCreateWithFlags(&c->solve_stream, hipStreamNonBlocking));
        if (!c->order_event) HIPCHK(hipEventCreateWithFlags(&c->order_event, hipEventDisableTiming));
        HIPCHK(hipEventRecord(c->order_event, user));
        HIPCHK(hipStreamWaitEvent(c->solve_stream, c->order_event, 0));
        c->s = c->solve_stream;
        eh_status st;
        if (c->o.mg_precision == 64) st = solve_impl<double>(c, (const c128*)b, (c128*)x, nrhs, tol, maxit, info);
        else st = solve_impl<float>(c, (const c128*)b, (c128*)x, nrhs, tol, maxit, info);
        HIPCHK(hipStreamSynchronize(c->s));
        c->s = user;
        return st;
    } catch (const StateError& e) {
        const hipError_t se = hipStreamSynchronize(c->s);   // steps may still be queued
        c->s = user;
        if (se != hipSuccess) return from_hip(c, HipError{se, "hipStreamSynchronize"});
        return fail(c, EH_ERR_STATE, e.msg);
    } catch (const HipError& e) {
        c->s = user;
        return from_hip(c, e);
    }
}

eh_status eh_block_solve(eh_ctx* c, int block, const void* f, void* x, int nrhs, double tol, int maxit,
                         eh_info* info) {
    EH_GUARD(c)
    if (block < 0 || block > c->dim || !f || !x || nrhs < 1 || !(tol > 0.0) || maxit < 0)
        return fail(c, EH_ERR_ARG, "invalid block solve arguments");
    try {
        eh_status st;
        if (c->o.mg_precision == 64) st = block_solve_impl<double>(c, block, (const c128*)f, (c128*)x, nrhs, tol, maxit, info);
        else st = block_solve_impl<float>(c, block, (const c128*)f, (c128*)x, nrhs, tol, maxit, info);
        HIPCHK(hipStreamSynchronize(c->s));
        return st;
    } catch (const StateError& e) {
        const hipError_t se = hipStreamSynchronize(c->s);
        if (se != hipSuccess) return from_hip(c, HipError{se, "hipStreamSynchronize"});
        return fail(c, EH_ERR_STATE, e.msg);
    } catch (const HipError& e) {
        return from_hip(c, e);
    }
}

eh_status eh_apply_Z(eh_ctx* c, const void* v, void* y, double tol, int maxit) {
    EH_GUARD(c)
    if (!v || !y || !(tol > 0.0) || maxit < 1) return fail(c, EH_ERR_ARG, "invalid Z arguments");
    try {
        eh_status st;
        if (c->o.mg_precision == 64) st = apply_Z_impl<double>(c, (const c128*)v, (c128*)y, tol, maxit);
        else st = apply_Z_impl<float>(c, (const c128*)v, (c128*)y, tol, maxit);
        HIPCHK(hipStreamSynchronize(c->s));
        return st;
    } catch (const StateError& e) {
        const hipError_t se = hipStreamSynchronize(c->s);
        if (se != hipSuccess) return from_hip(c, HipError{se, "hipStreamSynchronize"});
        return fail(c, EH_ERR_STATE, e.msg);
    } catch (const HipError& e) {
        return from_hip(c, e);
    }
}

eh_status eh_power_Z(eh_ctx* c, void* v, int iters, double tol, int maxit, double* est) {
    EH_GUARD(c)
    if (!v || iters < 1 || !est || !(tol > 0.0) || maxit < 1) return fail(c, EH_ERR_ARG, "invalid power method arguments");
    try {
        if (c->o.mg_precision == 64) return power_Z_impl<double>(c, (c128*)v, iters, tol, maxit, est);
        return power_Z_impl<float>(c, (c128*)v, iters, tol, maxit, est);
    } catch (const StateError& e) {
        const hipError_t se = hipStreamSynchronize(c->s);
        if (se != hipSuccess) return from_hip(c, HipError{se, "hipStreamSynchronize"});
        return fail(c, EH_ERR_STATE, e.msg);
    } catch (const HipError& e) {
        return from_hip(c, e);
    }
}

}  // extern "C"

#include "eh_grad_host.inc"
