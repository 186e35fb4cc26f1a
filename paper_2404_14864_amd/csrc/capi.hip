// C ABI of the library (declared in include/kfbi.h): domain lifecycle, the
// solve entry points and the time steppers of section 3.1.
//
// The steppers carry the paper's right-hand-side recurrences so that no
// discrete Laplacian of the numerical solution is ever formed; the same
// recurrence runs on the boundary trace with u = g there, which supplies
// f on Gamma for the jump conditions.
//   heat (eqs. 3.2-3.4, c u_t = lap u + s):  kappa = 2c/tau,
//        f = -(G + s^n + s^{n+1}),  G <- 2 kappa u^{n+1} + f
//        (G^n = kappa u^n + lap u^n; the paper's F^{n+1} = -f).
//   wave (eqs. 3.5-3.7, theta-scheme):  kappa = 1/(theta tau^2),
//        f = -F^{n+1},  F^{n+2} = (kappa/theta) u^{n+1}
//                                  - (1-2 theta)/theta F^{n+1} - F^n.
//   Schroedinger (Strang splitting after eq. 3.12):  kappa = 2i/tau,
//        u** = u* (1 - i beta)/(1 + i beta), beta = tau/2 (v + w|u*|^2),
//        f = -kappa u**,  u* <- 2 u^{n+1} - u**.
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>
#include <utility>

#include "kfbi_internal.h"

namespace kfbi {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }

int dalloc(kfbi_domain *d, void **p, size_t bytes) {
    if (bytes == 0) bytes = 256;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        set_error(std::string("hipMalloc: ") + hipGetErrorString(e));
        *p = nullptr;
        return KFBI_ENOMEM;
    }
    d->allocs.push_back(*p);
    d->bytes += bytes;
    return KFBI_OK;
}

size_t gmres_bytes(kfbi_domain *d);

int prof_begin(kfbi_domain *d) {
    if (!d->prof_on) return -1;
    kfbi_domain::ProfSlot s;
    hipEvent_t ev[2];
    for (int q = 0; q < 2; ++q) {
        if (!d->prof_pool.empty()) {
            ev[q] = d->prof_pool.back();
            d->prof_pool.pop_back();
        } else if (hipEventCreate(&ev[q]) != hipSuccess) {
            return -1;
        }
    }
    s.a = ev[0];
    s.b = ev[1];
    s.kind = -1;
    s.tag = d->prof_tag;
    s.bytes = 0.0;
    if (hipEventRecord(s.a, d->stream) != hipSuccess) return -1;
    d->prof_live.push_back(s);
    return (int)d->prof_live.size() - 1;
}

void prof_end(kfbi_domain *d, int slot, int kind, double bytes) {
    if (slot < 0 || slot >= (int)d->prof_live.size()) return;
    kfbi_domain::ProfSlot &s = d->prof_live[slot];
    s.kind = kind;
    s.bytes = bytes;
    (void)hipEventRecord(s.b, d->stream);
}

int prof_flush(kfbi_domain *d, int keep_tags_below, int keep_tag) {
    for (auto &s : d->prof_live) {
        KFBI_HIP(hipEventSynchronize(s.b));
        if (s.kind >= 0 && (s.tag < 0 || s.tag < keep_tags_below || s.tag == keep_tag)) {
            float ms = 0.f;
            KFBI_HIP(hipEventElapsedTime(&ms, s.a, s.b));
            d->prof_count[s.kind] += 1;
            d->prof_ms[s.kind] += ms;
            d->prof_bytes[s.kind] += s.bytes;
        }
        d->prof_pool.push_back(s.a);
        d->prof_pool.push_back(s.b);
    }
    d->prof_live.clear();
    return KFBI_OK;
}

namespace {

// out = sum_q c_q x_q over up to four operands (null operands are skipped)
template <class T>
__global__ void k_lin4(int n, T *out, T c0, const T *x0, T c1, const T *x1, T c2, const T *x2, T c3,
                       const T *x3) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    T acc = zero<T>();
    if (x0) acc += c0 * x0[i];
    if (x1) acc += c1 * x1[i];
    if (x2) acc += c2 * x2[i];
    if (x3) acc += c3 * x3[i];
    out[i] = acc;
}

// Schroedinger B-step in closed form (the Crank-Nicolson step of eq. 3.10
// over tau), in place on u (u* -> u**), and f = -kappa u** with
// kappa = i kim (2i/tau for Strang, i/tau for Godunov), on the grid (indices
// below ng) and on Gamma (the next nb) in one launch
__global__ void k_schr_b(int ng, int nb, cd *ugr, const double *vgr, cd *fgr, cd *uga, const double *vga, cd *fga,
                         double w, double tau, double kim) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool grid = i < ng;
    if (!grid) i -= ng;
    if (i >= (grid ? ng : nb)) return;
    cd *u = grid ? ugr : uga;
    const double *v = grid ? vgr : vga;
    cd *f = grid ? fgr : fga;
    cd us = u[i];
    double beta = 0.5 * tau * ((v ? v[i] : 0.0) + w * abs2(us));
    cd uss = us * make_cd(1.0, -beta) / make_cd(1.0, beta);
    u[i] = uss;
    // -(i kim) uss
    f[i] = make_cd(kim * uss.y, -kim * uss.x);
}

template <class T>
int lin4(kfbi_domain *d, int n, void *out, T c0, const void *x0, T c1 = zero<T>(), const void *x1 = nullptr,
         T c2 = zero<T>(), const void *x2 = nullptr, T c3 = zero<T>(), const void *x3 = nullptr) {
    k_lin4<T><<<(n + 255) / 256, 256, 0, d->stream>>>(n, (T *)out, c0, (const T *)x0, c1, (const T *)x1, c2,
                                                       (const T *)x2, c3, (const T *)x3);
    KFBI_CHECK_LAUNCH();
    return KFBI_OK;
}

// the same combination on the grid and on Gamma in one launch: indices
// below ng address the grid arrays, the next nb the Gamma arrays
template <class T>
struct Lin4Set {
    T *out;
    const T *x0, *x1, *x2, *x3;
};

template <class T>
__global__ void k_lin4_pair(int ng, int nb, Lin4Set<T> g, Lin4Set<T> b, T c0, T c1, T c2, T c3) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool grid = i < ng;
    if (!grid) i -= ng;
    if (i >= (grid ? ng : nb)) return;
    const Lin4Set<T> &P = grid ? g : b;
    T acc = zero<T>();
    if (P.x0) acc += c0 * P.x0[i];
    if (P.x1) acc += c1 * P.x1[i];
    if (P.x2) acc += c2 * P.x2[i];
    if (P.x3) acc += c3 * P.x3[i];
    P.out[i] = acc;
}

template <class T>
int lin4_pair(kfbi_domain *d, int ng, int nb, Lin4Set<T> g, Lin4Set<T> b, T c0, T c1 = zero<T>(),
              T c2 = zero<T>(), T c3 = zero<T>()) {
    k_lin4_pair<T><<<(ng + nb + 255) / 256, 256, 0, d->stream>>>(ng, nb, g, b, c0, c1, c2, c3);
    KFBI_CHECK_LAUNCH();
    return KFBI_OK;
}

template <class T>
Lin4Set<T> lset(void *out, const void *x0, const void *x1 = nullptr, const void *x2 = nullptr,
                const void *x3 = nullptr) {
    return Lin4Set<T>{(T *)out, (const T *)x0, (const T *)x1, (const T *)x2, (const T *)x3};
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

}  // namespace
}  // namespace kfbi

using namespace kfbi;

struct kfbi_stepper {
    kfbi_domain *dom = nullptr;
    int eq = 0;
    kfbi_step_params p{};
    double kre = 0, kim = 0;
    bool initialized = false;
    std::vector<void *> allocs;
    // state (grid, Gamma)
    void *A = nullptr, *Ag = nullptr;   // heat: G;  wave: F^{n+1};  schr: u*
    void *B = nullptr, *Bg = nullptr;   // wave: F^n
    void *f = nullptr, *fg = nullptr;   // right-hand side of the current solve
    void *phi = nullptr;                // warm start / density
    void *tr = nullptr;                 // Neumann: U+ on Gamma of the last step
    void *v = nullptr, *vg = nullptr;   // Schroedinger: copies of the potential
};

// The B-step of a Schroedinger step in place on the carried state (u* for
// Strang, u^n for Godunov), with the right-hand side f = -kappa u** of the
// A-step's solve, on the grid and on Gamma.
static int schr_b_step(kfbi_stepper *s) {
    kfbi_domain *d = s->dom;
    const int ng = (d->M + 1) * (d->M + 1), Nb = d->Nb;
    k_schr_b<<<(ng + Nb + 255) / 256, 256, 0, d->stream>>>(ng, Nb, (cd *)s->A, (const double *)s->v, (cd *)s->f,
                                                          (cd *)s->Ag, (const double *)s->vg, (cd *)s->fg, s->p.w,
                                                          s->p.tau, s->kim);
    KFBI_CHECK_LAUNCH();
    return KFBI_OK;
}

// The carried state after the A-step's solve u^{n+1} (trace tr on Gamma).
static int schr_state_update(kfbi_stepper *s, const void *u, const void *tr) {
    kfbi_domain *d = s->dom;
    const int ng = (d->M + 1) * (d->M + 1), Nb = d->Nb;
    if (s->p.split == KFBI_SPLIT_GODUNOV) {
        // the next B-step acts on u^{n+1} itself
        return lin4_pair<cd>(d, ng, Nb, lset<cd>(s->A, u), lset<cd>(s->Ag, tr), make_cd(1.0, 0.0));
    }
    // u* of the next step, u^{n+1} - i tau/2 lap u^{n+1} = 2 u^{n+1} - u** (eq. 3.12)
    const cd two = make_cd(2.0, 0.0), m1 = make_cd(-1.0, 0.0);
    return lin4_pair<cd>(d, ng, Nb, lset<cd>(s->A, u, s->A), lset<cd>(s->Ag, tr, s->Ag), two, m1);
}

extern "C" {

const char *kfbi_last_error(void) { return g_err.c_str(); }

int kfbi_domain_create(const kfbi_domain_desc *desc, kfbi_domain **out) {
    if (!desc || !out) { set_error("null argument"); return KFBI_EINVAL; }
    *out = nullptr;
    const kfbi_domain_desc &D = *desc;
    if (!is_pow2(D.M) || D.M < 16 || D.M > 2048) {
        set_error("M must be a power of two in [16, 2048]");
        return KFBI_EINVAL;
    }
    if (D.Nb < 8 || D.Nb > 16384) { set_error("Nb must be in [8, 16384]"); return KFBI_EDOMAIN; }
    if (!(D.L > 0)) { set_error("L must be positive"); return KFBI_EINVAL; }
    if (D.kind < 0 || D.kind > 2) { set_error("unknown curve kind"); return KFBI_EINVAL; }
    if (D.kind == KFBI_CURVE_DISK && !(D.R > 0)) { set_error("disk radius must be positive"); return KFBI_EINVAL; }
    if (D.kind == KFBI_CURVE_ELLIPSE && !(D.a > 0 && D.b > 0)) { set_error("ellipse axes must be positive"); return KFBI_EINVAL; }
    if (D.kind == KFBI_CURVE_STAR && !(D.r0 > 0 && D.amp >= 0 && D.amp < D.r0 && D.lobes >= 1 && D.lobes <= 64)) {
        set_error("star needs r0 > amp >= 0 and 1 <= lobes <= 64");
        return KFBI_EINVAL;
    }
    if (D.scalar != KFBI_REAL && D.scalar != KFBI_COMPLEX) { set_error("bad scalar type"); return KFBI_EINVAL; }
    kfbi_domain *d = new kfbi_domain();
    d->desc = D;
    d->M = D.M;
    d->Nb = D.Nb;
    d->n = D.M - 1;
    d->L = D.L;
    d->h = (2.0 * D.L) / D.M;
    d->cplx = D.scalar == KFBI_COMPLEX;
    d->stream = (hipStream_t)D.stream;
    int st = build_domain(d);
    if (st == KFBI_OK) {
        // set-up of the no-allocation grid solve: look up this device's
        // scratch array once (a failure is reported by that call itself)
        void *scr = nullptr;
        if (noalloc_scratch(d->stream, &scr) != KFBI_OK) set_error("");
    }
    if (st == KFBI_OK) {
        const size_t es = elem_size(d), n = d->n, Nb = d->Nb;
        const size_t nodes = (size_t)(d->M + 1) * (d->M + 1);
        (void)nodes;
        int s2 = KFBI_OK;
        if (s2 == KFBI_OK) s2 = dalloc(d, &d->rhat, n * n * es);
        if (s2 == KFBI_OK) s2 = dalloc(d, &d->uhat, n * n * es);
        if (s2 == KFBI_OK) s2 = dalloc(d, &d->corr, (size_t)d->n_irr * es);
        if (s2 == KFBI_OK) s2 = dalloc(d, &d->corr_f, (size_t)d->n_irr * es);
        if (s2 == KFBI_OK) s2 = dalloc(d, &d->ust, 6 * Nb * es);
        if (s2 == KFBI_OK) s2 = dalloc(d, &d->etab, n * n * es);
        if (s2 == KFBI_OK) s2 = dalloc(d, &d->elim, n * es);
        if (s2 == KFBI_OK) s2 = dalloc(d, (void **)&d->tconv, n * sizeof(int32_t));
        if (s2 == KFBI_OK) { d->gm_bytes = gmres_bytes(d); s2 = dalloc(d, &d->gm, d->gm_bytes); }
        st = s2;
    }
    if (st != KFBI_OK) {
        std::string keep = g_err;
        kfbi_domain_destroy(d);
        g_err = keep;
        return st;
    }
    *out = d;
    return KFBI_OK;
}

int kfbi_profile_enable(kfbi_domain *d, int32_t on) {
    if (!d) { set_error("null domain"); return KFBI_EINVAL; }
    KFBI_TRY(prof_flush(d, 0));
    for (int k = 0; k < KFBI_K_COUNT; ++k) {
        d->prof_count[k] = 0;
        d->prof_ms[k] = 0.0;
        d->prof_bytes[k] = 0.0;
    }
    d->prof_on = on != 0;
    return KFBI_OK;
}

int kfbi_batch_create(kfbi_domain *const *doms, int32_t n, kfbi_batch **out) {
    return batch_create(doms, n, out);
}

int kfbi_batch_destroy(kfbi_batch *b) {
    batch_destroy(b);
    return KFBI_OK;
}

int kfbi_batch_helmholtz(kfbi_batch *b, const double *kappa_re, const double *kappa_im, const void *const *f_grid,
                         const void *const *f_gamma, const void *const *g_gamma, void *const *u_grid_out,
                         void *const *phi_inout, const kfbi_solve_opts *opts, kfbi_solve_stats *stats) {
    return batch_helmholtz(b, kappa_re, kappa_im, f_grid, f_gamma, g_gamma, u_grid_out, phi_inout, opts, stats);
}

int kfbi_batch_step(kfbi_batch *b, kfbi_stepper *const *st, const uint8_t *active, const void *const *g_next,
                    const void *const *src_grid, const void *const *src_gamma, void *const *u_out,
                    const kfbi_solve_opts *opts, kfbi_solve_stats *stats) {
    if (!b || !st || !g_next || !u_out) { set_error("null argument"); return KFBI_EINVAL; }
    const int n = batch_size(b);
    const bool cplx = batch_complex(b);
    auto on = [&](int q) { return !active || active[q] != 0; };
    std::vector<double> kap(n, 0.0), kapi(n, 0.0);
    std::vector<const void *> f(n, nullptr), fg(n, nullptr), g(n, nullptr);
    std::vector<void *> u(n, nullptr), phi(n, nullptr);
    for (int q = 0; q < n; ++q) {
        if (!on(q)) continue;
        kfbi_stepper *s = st[q];
        if (!s || !g_next[q] || !u_out[q]) { set_error("null stepper or array of an active member"); return KFBI_EINVAL; }
        if (s->dom != batch_domain(b, q)) { set_error("stepper is not on the batch member's domain"); return KFBI_EINVAL; }
        if (!s->initialized) { set_error("batched steps take initialised steppers"); return KFBI_EINVAL; }
        if (cplx ? s->eq != KFBI_SCHRODINGER : (s->eq != KFBI_HEAT && s->eq != KFBI_WAVE)) {
            set_error("batched steps take heat or wave steppers (real batch) or Schroedinger steppers "
                      "(complex batch)");
            return KFBI_EINVAL;
        }
        if (s->p.bc != KFBI_BC_DIRICHLET) {
            set_error("batched steps take Dirichlet steppers only");
            return KFBI_ENOTSUP;
        }
    }
    // right-hand sides of the members' solves (as kfbi_step_heat / kfbi_step_wave)
    for (int q = 0; q < n; ++q) {
        if (!on(q)) continue;
        kfbi_stepper *s = st[q];
        kfbi_domain *d = s->dom;
        const int ng = (d->M + 1) * (d->M + 1), Nb = d->Nb;
        if (s->eq == KFBI_HEAT) {
            const void *sg = src_grid ? src_grid[q] : nullptr, *sgg = src_gamma ? src_gamma[q] : nullptr;
            KFBI_TRY(lin4_pair<double>(d, ng, Nb, lset<double>(s->f, s->A, sg), lset<double>(s->fg, s->Ag, sgg), -1.0,
                                       -1.0));
        } else if (s->eq == KFBI_WAVE) {
            KFBI_TRY(lin4_pair<double>(d, ng, Nb, lset<double>(s->f, s->A), lset<double>(s->fg, s->Ag), -1.0));
        } else {
            KFBI_TRY(schr_b_step(s));
        }
        kap[q] = s->kre;
        kapi[q] = s->kim;
        f[q] = s->f;
        fg[q] = s->fg;
        g[q] = g_next[q];
        u[q] = u_out[q];
        phi[q] = s->phi;
    }
    const int rc = batch_helmholtz(b, kap.data(), cplx ? kapi.data() : nullptr, f.data(), fg.data(), g.data(),
                                   u.data(), phi.data(), opts, stats, active);
    if (rc != KFBI_OK && rc != KFBI_ENOCONV) return rc;
    // state updates (as the single steps)
    for (int q = 0; q < n; ++q) {
        if (!on(q)) continue;
        kfbi_stepper *s = st[q];
        kfbi_domain *d = s->dom;
        const int ng = (d->M + 1) * (d->M + 1), Nb = d->Nb;
        if (s->eq == KFBI_HEAT) {
            KFBI_TRY(lin4_pair<double>(d, ng, Nb, lset<double>(s->A, u_out[q], s->f),
                                       lset<double>(s->Ag, g_next[q], s->fg), 2.0 * s->kre, 1.0));
        } else if (s->eq == KFBI_SCHRODINGER) {
            KFBI_TRY(schr_state_update(s, u_out[q], g_next[q]));
        } else {
            const double th = s->p.theta, c1 = (1.0 - 2.0 * th) / th, a = s->kre / th;
            KFBI_TRY(lin4_pair<double>(d, ng, Nb, lset<double>(s->B, u_out[q], s->A, s->B),
                                       lset<double>(s->Bg, g_next[q], s->Ag, s->Bg), a, -c1, -1.0));
            std::swap(s->A, s->B);
            std::swap(s->Ag, s->Bg);
        }
    }
    if (rc == KFBI_ENOCONV) set_error("GMRES reached max_iter before the tolerance for a batch member");
    return rc;
}

int kfbi_batch_tuning(const kfbi_batch *b, int32_t cap, int32_t *rows, double *us, int32_t *n_rows) {
    return batch_tuning(b, cap, rows, us, n_rows);
}

int kfbi_profile_replay(kfbi_domain *d, int32_t kind, int32_t reps, double *avg_ms, double *bytes_per_launch) {
    if (!d || !avg_ms || !bytes_per_launch) { set_error("null argument"); return KFBI_EINVAL; }
    if (reps < 1 || reps > 100000) { set_error("reps must be in 1..100000"); return KFBI_EINVAL; }
    if (kind == KFBI_K_ARNOLDI) return replay_slot(d, reps, avg_ms, bytes_per_launch);
    if (kind != KFBI_K_TRIDIAG_SPARSE && kind != KFBI_K_TRIDIAG_DENSE && kind != KFBI_K_EVAL_NODES &&
        kind != KFBI_K_CORRECTIONS) {
        set_error("replay supports the tridiagonal, stencil-evaluation, corrections and control kernels only");
        return KFBI_EINVAL;
    }
    if (kind == KFBI_K_CORRECTIONS && !d->op_merged) {
        set_error("the corrections replay needs the merged operators of the device-driven schedule");
        return KFBI_ENOTSUP;
    }
    if (!d->coef_valid) { set_error("no solve has run on this domain"); return KFBI_EINVAL; }
    const void *phi = gmres_last_density(d);
    if (!phi) { set_error("no solve has run on this domain"); return KFBI_EINVAL; }
    // the sparse form replays the grid solve of the last density's
    // corrections (formed once here, outside the timed launches)
    if (kind == KFBI_K_TRIDIAG_SPARSE && d->op_merged) KFBI_TRY(corrections_of_density(d, phi, d->corr, nullptr));
    auto launch = [&]() -> int {
        if (kind == KFBI_K_TRIDIAG_SPARSE) return tridiag_solve(d, nullptr, d->corr, d->uhat);
        if (kind == KFBI_K_TRIDIAG_DENSE) return tridiag_solve(d, d->rhat, d->corr, d->uhat);
        if (kind == KFBI_K_CORRECTIONS) return corrections_of_density(d, phi, d->corr, nullptr);
        return eval_stencil_nodes(d, d->uhat, d->ust);
    };
    // algorithmic bytes of one launch, through the profiler's own accounting
    KFBI_TRY(prof_flush(d, 1 << 30));
    const bool was_on = d->prof_on;
    const int64_t c0 = d->prof_count[kind];
    const double m0 = d->prof_ms[kind], b0 = d->prof_bytes[kind];
    d->prof_on = true;
    const int st = launch();
    d->prof_on = was_on;
    KFBI_TRY(st);
    KFBI_TRY(prof_flush(d, 1 << 30));
    *bytes_per_launch = d->prof_bytes[kind] - b0;
    d->prof_count[kind] = c0;
    d->prof_ms[kind] = m0;
    d->prof_bytes[kind] = b0;
    // timing: reps launches between two events
    hipEvent_t e0, e1;
    KFBI_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) { hipEventDestroy(e0); set_error("hipEventCreate failed"); return KFBI_EDEVICE; }
    int rc = KFBI_OK;
    const bool was_on2 = d->prof_on;
    d->prof_on = false;
    if (hipEventRecord(e0, d->stream) != hipSuccess) rc = KFBI_EDEVICE;
    for (int r = 0; r < reps && rc == KFBI_OK; ++r) rc = launch();
    if (rc == KFBI_OK && hipEventRecord(e1, d->stream) != hipSuccess) rc = KFBI_EDEVICE;
    if (rc == KFBI_OK && hipEventSynchronize(e1) != hipSuccess) rc = KFBI_EDEVICE;
    float ms = 0.f;
    if (rc == KFBI_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = KFBI_EDEVICE;
    d->prof_on = was_on2;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc == KFBI_EDEVICE) set_error("HIP event or launch failure during replay");
    if (rc != KFBI_OK) return rc;
    *avg_ms = ms / reps;
    return KFBI_OK;
}

int kfbi_profile_read(kfbi_domain *d, kfbi_kernel_prof *out) {
    if (!d || !out) { set_error("null argument"); return KFBI_EINVAL; }
    KFBI_TRY(prof_flush(d, 1 << 30));
    for (int k = 0; k < KFBI_K_COUNT; ++k) {
        out[k].launches = d->prof_count[k];
        out[k].total_ms = d->prof_ms[k];
        out[k].bytes = d->prof_bytes[k];
    }
    return KFBI_OK;
}

int kfbi_domain_destroy(kfbi_domain *d) {
    if (!d) return KFBI_OK;
    if (d->stream) hipStreamSynchronize(d->stream);
    else hipDeviceSynchronize();
    for (auto &s : d->prof_live) { hipEventDestroy(s.a); hipEventDestroy(s.b); }
    for (hipEvent_t e : d->prof_pool) hipEventDestroy(e);
    if (d->mirror_host) hipHostFree(d->mirror_host);
    if (d->ev0) hipEventDestroy(d->ev0);
    if (d->ev1) hipEventDestroy(d->ev1);
    for (void *p : d->allocs) hipFree(p);
    delete d;
    return KFBI_OK;
}

int kfbi_domain_get_info(const kfbi_domain *d, kfbi_domain_info *out) {
    if (!d || !out) { set_error("null argument"); return KFBI_EINVAL; }
    memset(out, 0, sizeof(*out));
    out->M = d->M;
    out->Nb = d->Nb;
    out->L = d->L;
    out->h = d->h;
    out->n_inside = d->n_inside;
    out->n_irregular = d->n_irr;
    out->n_edges = d->n_edges;
    out->scalar = d->cplx ? KFBI_COMPLEX : KFBI_REAL;
    out->device_bytes = d->bytes;
    out->device_bytes_max = d->bytes + operators_bytes_pending(d) + low_tables_bytes_pending(d);
    return KFBI_OK;
}

int kfbi_domain_copy_classification(const kfbi_domain *d, uint8_t *host_out) {
    if (!d || !host_out) { set_error("null argument"); return KFBI_EINVAL; }
    size_t nodes = (size_t)(d->M + 1) * (d->M + 1);
    KFBI_HIP(hipMemcpyAsync(host_out, d->flags, nodes, hipMemcpyDeviceToHost, d->stream));
    KFBI_HIP(hipStreamSynchronize(d->stream));
    return KFBI_OK;
}

int kfbi_domain_copy_boundary(const kfbi_domain *d, double *host_out) {
    if (!d || !host_out) { set_error("null argument"); return KFBI_EINVAL; }
    std::vector<Colloc> c(d->Nb);
    KFBI_HIP(hipMemcpyAsync(c.data(), d->col, d->Nb * sizeof(Colloc), hipMemcpyDeviceToHost, d->stream));
    KFBI_HIP(hipStreamSynchronize(d->stream));
    for (int k = 0; k < d->Nb; ++k) {
        host_out[2 * k] = c[k].x;
        host_out[2 * k + 1] = c[k].y;
    }
    return KFBI_OK;
}

int kfbi_domain_copy_normals(const kfbi_domain *d, double *host_out) {
    if (!d || !host_out) { set_error("null argument"); return KFBI_EINVAL; }
    std::vector<Colloc> c(d->Nb);
    KFBI_HIP(hipMemcpyAsync(c.data(), d->col, d->Nb * sizeof(Colloc), hipMemcpyDeviceToHost, d->stream));
    KFBI_HIP(hipStreamSynchronize(d->stream));
    for (int k = 0; k < d->Nb; ++k) {
        host_out[2 * k] = c[k].fr.ty;
        host_out[2 * k + 1] = -c[k].fr.tx;
    }
    return KFBI_OK;
}

int kfbi_domain_copy_edges(const kfbi_domain *d, int32_t *pq, double *xyt) {
    if (!d || !pq || !xyt) { set_error("null argument"); return KFBI_EINVAL; }
    std::vector<Edge> e(d->n_edges);
    KFBI_HIP(hipMemcpyAsync(e.data(), d->edges, d->n_edges * sizeof(Edge), hipMemcpyDeviceToHost, d->stream));
    KFBI_HIP(hipStreamSynchronize(d->stream));
    for (int q = 0; q < d->n_edges; ++q) {
        pq[2 * q] = e[q].p_in;
        pq[2 * q + 1] = e[q].q_out;
        xyt[3 * q] = e[q].X;
        xyt[3 * q + 1] = e[q].Y;
        xyt[3 * q + 2] = e[q].theta;
    }
    return KFBI_OK;
}

static int check_kappa(const kfbi_domain *d, double kim) {
    if (!d->cplx && kim != 0.0) {
        set_error("complex kappa needs a complex domain");
        return KFBI_EINVAL;
    }
    return KFBI_OK;
}

int kfbi_grid_solve(kfbi_domain *d, double kre, double kim, const void *rhs, void *u_out) {
    if (!d || !rhs || !u_out) { set_error("null argument"); return KFBI_EINVAL; }
    KFBI_TRY(check_kappa(d, kim));
    KFBI_TRY(dst_rows_dense(d, rhs, false, d->rhat));
    KFBI_TRY(ensure_coefficients(d, kre, kim));
    KFBI_TRY(tridiag_solve(d, d->rhat, nullptr, d->uhat));
    KFBI_TRY(idst_rows_dense(d, d->uhat, u_out));
    return KFBI_OK;
}

int kfbi_interface_apply(kfbi_domain *d, double kre, double kim, const void *f_grid, const void *f_gamma,
                         const void *phi, void *u_grid_out, void *uplus_out) {
    if (!d) { set_error("null domain"); return KFBI_EINVAL; }
    KFBI_TRY(check_kappa(d, kim));
    if (f_grid && !f_gamma) { set_error("f_gamma is required when f_grid is given"); return KFBI_EINVAL; }
    KFBI_TRY(interface_solve(d, kre, kim, f_grid, f_gamma, phi, u_grid_out, uplus_out, false));
    return KFBI_OK;
}

int kfbi_helmholtz_solve(kfbi_domain *d, double kre, double kim, const void *f_grid, const void *f_gamma,
                         const void *g_gamma, void *u_grid_out, void *phi_inout, const kfbi_solve_opts *opts,
                         kfbi_solve_stats *stats) {
    if (!d || !g_gamma) { set_error("null argument"); return KFBI_EINVAL; }
    KFBI_TRY(check_kappa(d, kim));
    return helmholtz_solve(d, kre, kim, f_grid, f_gamma, g_gamma, u_grid_out, phi_inout, opts, stats);
}

int kfbi_neumann_solve(kfbi_domain *d, double kre, double kim, const void *f_grid, const void *f_gamma,
                       const void *gn_gamma, void *u_grid_out, void *psi_inout, void *trace_out,
                       const kfbi_solve_opts *opts, kfbi_solve_stats *stats) {
    if (!d || !gn_gamma) { set_error("null argument"); return KFBI_EINVAL; }
    KFBI_TRY(check_kappa(d, kim));
    if (kre == 0.0 && kim == 0.0) {
        set_error("the Neumann problem needs kappa != 0 (for kappa = 0 its solution is not unique)");
        return KFBI_EINVAL;
    }
    return helmholtz_solve(d, kre, kim, f_grid, f_gamma, gn_gamma, u_grid_out, psi_inout, opts, stats, 1,
                           trace_out);
}

// ---------------------------------------------------------------------------
// steppers
// ---------------------------------------------------------------------------
static int st_alloc(kfbi_stepper *s, void **p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) { set_error("hipMalloc failed for stepper state"); return KFBI_ENOMEM; }
    s->allocs.push_back(*p);
    return KFBI_OK;
}

int kfbi_stepper_create(kfbi_domain *d, int32_t eq, const kfbi_step_params *p, kfbi_stepper **out) {
    if (!d || !p || !out) { set_error("null argument"); return KFBI_EINVAL; }
    *out = nullptr;
    if (eq < 0 || eq > 2) { set_error("unknown equation"); return KFBI_EINVAL; }
    if (!(p->tau > 0)) { set_error("tau must be positive"); return KFBI_EINVAL; }
    if ((eq == KFBI_SCHRODINGER) != d->cplx) {
        set_error("Schroedinger needs a complex domain; heat and wave a real one");
        return KFBI_EINVAL;
    }
    if (p->bc != KFBI_BC_DIRICHLET && p->bc != KFBI_BC_NEUMANN) {
        set_error("unknown boundary condition");
        return KFBI_EINVAL;
    }
    kfbi_stepper *s = new kfbi_stepper();
    s->dom = d;
    s->eq = eq;
    s->p = *p;
    if (eq == KFBI_HEAT) {
        double c = p->diffusivity > 0 ? p->diffusivity : 1.0;
        s->kre = 2.0 * c / p->tau;
    } else if (eq == KFBI_WAVE) {
        if (!(p->theta > 0 && p->theta <= 0.5)) { delete s; set_error("theta must be in (0, 1/2]"); return KFBI_EINVAL; }
        s->kre = 1.0 / (p->theta * p->tau * p->tau);
    } else {
        if (p->split != KFBI_SPLIT_STRANG && p->split != KFBI_SPLIT_GODUNOV) {
            delete s;
            set_error("unknown splitting");
            return KFBI_EINVAL;
        }
        s->kre = 0.0;
        s->kim = (p->split == KFBI_SPLIT_GODUNOV ? 1.0 : 2.0) / p->tau;
    }
    const size_t es = elem_size(d), nodes = (size_t)(d->M + 1) * (d->M + 1), Nb = d->Nb;
    int st = KFBI_OK;
    if (st == KFBI_OK) st = st_alloc(s, &s->A, nodes * es);
    if (st == KFBI_OK) st = st_alloc(s, &s->Ag, Nb * es);
    if (st == KFBI_OK) st = st_alloc(s, &s->B, nodes * es);
    if (st == KFBI_OK) st = st_alloc(s, &s->Bg, Nb * es);
    if (st == KFBI_OK) st = st_alloc(s, &s->f, nodes * es);
    if (st == KFBI_OK) st = st_alloc(s, &s->fg, Nb * es);
    if (st == KFBI_OK) st = st_alloc(s, &s->phi, Nb * es);
    if (st == KFBI_OK && p->bc == KFBI_BC_NEUMANN) st = st_alloc(s, &s->tr, Nb * es);
    // the potential is copied: the caller's arrays need not outlive the call
    if (st == KFBI_OK && eq == KFBI_SCHRODINGER && p->v_grid) {
        st = st_alloc(s, &s->v, nodes * sizeof(double));
        if (st == KFBI_OK &&
            hipMemcpyAsync(s->v, p->v_grid, nodes * sizeof(double), hipMemcpyDeviceToDevice, d->stream) != hipSuccess)
            st = KFBI_EDEVICE;
    }
    if (st == KFBI_OK && eq == KFBI_SCHRODINGER && p->v_gamma) {
        st = st_alloc(s, &s->vg, Nb * sizeof(double));
        if (st == KFBI_OK &&
            hipMemcpyAsync(s->vg, p->v_gamma, Nb * sizeof(double), hipMemcpyDeviceToDevice, d->stream) != hipSuccess)
            st = KFBI_EDEVICE;
    }
    if (st == KFBI_OK && (s->v || s->vg) && hipStreamSynchronize(d->stream) != hipSuccess) st = KFBI_EDEVICE;
    s->p.v_grid = s->v;
    s->p.v_gamma = s->vg;
    // every state buffer starts at zero (the checkpoint of a stepper is then
    // a function of its steps alone, also for buffers its equation leaves unused)
    void *zero_bufs[5] = {s->A, s->Ag, s->B, s->Bg, s->phi};
    const size_t zero_sizes[5] = {nodes * es, Nb * es, nodes * es, Nb * es, Nb * es};
    for (int q = 0; q < 5 && st == KFBI_OK; ++q)
        if (hipMemsetAsync(zero_bufs[q], 0, zero_sizes[q], d->stream) != hipSuccess) st = KFBI_EDEVICE;
    if (st != KFBI_OK) { kfbi_stepper_destroy(s); return st; }
    *out = s;
    return KFBI_OK;
}

namespace {
struct StateHeader {
    uint32_t magic, version;
    int32_t eq, M, Nb, cplx, initialized, bc;
    double tau, kre, kim, pad2;
};
static_assert(sizeof(StateHeader) == 64, "state header is 64 bytes");
constexpr uint32_t kStateMagic = 0x5346424bu;  // "KBFS"

size_t state_bytes(const kfbi_stepper *s) {
    const kfbi_domain *d = s->dom;
    const size_t es = elem_size(d), nodes = (size_t)(d->M + 1) * (d->M + 1), Nb = d->Nb;
    return sizeof(StateHeader) + 2 * nodes * es + 3 * Nb * es;
}
}  // namespace

int kfbi_stepper_state_bytes(const kfbi_stepper *s, uint64_t *bytes) {
    if (!s || !bytes) { set_error("null argument"); return KFBI_EINVAL; }
    *bytes = state_bytes(s);
    return KFBI_OK;
}

int kfbi_stepper_get_state(kfbi_stepper *s, void *dst, uint64_t bytes) {
    if (!s || !dst) { set_error("null argument"); return KFBI_EINVAL; }
    if (bytes < state_bytes(s)) { set_error("state buffer too small"); return KFBI_EINVAL; }
    kfbi_domain *d = s->dom;
    const size_t es = elem_size(d), nodes = (size_t)(d->M + 1) * (d->M + 1), Nb = d->Nb;
    StateHeader h{};
    h.magic = kStateMagic;
    h.version = 1;
    h.eq = s->eq;
    h.M = d->M;
    h.Nb = d->Nb;
    h.cplx = d->cplx ? 1 : 0;
    h.initialized = s->initialized ? 1 : 0;
    h.bc = s->p.bc;
    h.tau = s->p.tau;
    h.kre = s->kre;
    h.kim = s->kim;
    char *p = (char *)dst;
    KFBI_HIP(hipMemcpyAsync(p, &h, sizeof(h), hipMemcpyHostToDevice, d->stream));
    p += sizeof(h);
    const void *parts[5] = {s->A, s->B, s->Ag, s->Bg, s->phi};
    const size_t sizes[5] = {nodes * es, nodes * es, Nb * es, Nb * es, Nb * es};
    for (int q = 0; q < 5; ++q) {
        KFBI_HIP(hipMemcpyAsync(p, parts[q], sizes[q], hipMemcpyDeviceToDevice, d->stream));
        p += sizes[q];
    }
    KFBI_HIP(hipStreamSynchronize(d->stream));
    return KFBI_OK;
}

int kfbi_stepper_set_state(kfbi_stepper *s, const void *src, uint64_t bytes) {
    if (!s || !src) { set_error("null argument"); return KFBI_EINVAL; }
    if (bytes < state_bytes(s)) { set_error("state buffer too small"); return KFBI_EINVAL; }
    kfbi_domain *d = s->dom;
    const size_t es = elem_size(d), nodes = (size_t)(d->M + 1) * (d->M + 1), Nb = d->Nb;
    StateHeader h{};
    KFBI_HIP(hipMemcpyAsync(&h, src, sizeof(h), hipMemcpyDeviceToHost, d->stream));
    KFBI_HIP(hipStreamSynchronize(d->stream));
    if (h.magic != kStateMagic || h.version != 1) { set_error("not a stepper state blob"); return KFBI_EINVAL; }
    if (h.eq != s->eq || h.M != d->M || h.Nb != d->Nb || h.cplx != (d->cplx ? 1 : 0) || h.kre != s->kre ||
        h.kim != s->kim || h.bc != s->p.bc) {
        set_error("state blob belongs to a different stepper configuration");
        return KFBI_EINVAL;
    }
    const char *p = (const char *)src + sizeof(h);
    void *parts[5] = {s->A, s->B, s->Ag, s->Bg, s->phi};
    const size_t sizes[5] = {nodes * es, nodes * es, Nb * es, Nb * es, Nb * es};
    for (int q = 0; q < 5; ++q) {
        KFBI_HIP(hipMemcpyAsync(parts[q], p, sizes[q], hipMemcpyDeviceToDevice, d->stream));
        p += sizes[q];
    }
    KFBI_HIP(hipStreamSynchronize(d->stream));
    s->initialized = h.initialized != 0;
    return KFBI_OK;
}

int kfbi_stepper_destroy(kfbi_stepper *s) {
    if (!s) return KFBI_OK;
    if (s->dom && s->dom->stream) hipStreamSynchronize(s->dom->stream);
    else hipDeviceSynchronize();
    for (void *p : s->allocs) hipFree(p);
    delete s;
    return KFBI_OK;
}

int kfbi_stepper_init(kfbi_stepper *s, const void *u0, const void *lap0, const void *u0g, const void *lap0g,
                      const void *um1, const void *lapm1, const void *um1g, const void *lapm1g) {
    if (!s || !u0 || !lap0 || !u0g || !lap0g) { set_error("u0 and lap u0 on grid and Gamma are required"); return KFBI_EINVAL; }
    kfbi_domain *d = s->dom;
    const int ng = (d->M + 1) * (d->M + 1), Nb = d->Nb;
    if (s->eq == KFBI_HEAT) {
        // G^0 = kappa u^0 + lap u^0
        KFBI_TRY(lin4<double>(d, ng, s->A, s->kre, u0, 1.0, lap0));
        KFBI_TRY(lin4<double>(d, Nb, s->Ag, s->kre, u0g, 1.0, lap0g));
    } else if (s->eq == KFBI_WAVE) {
        if (!um1 || !lapm1 || !um1g || !lapm1g) { set_error("wave needs u^{-1} and lap u^{-1}"); return KFBI_EINVAL; }
        const double k = s->kre, th = s->p.theta, c1 = (1.0 - 2.0 * th) / th;
        // F^1 = kappa (2 u^0 - u^{-1}) + c1 lap u^0 + lap u^{-1};  F^0 = kappa u^0 - lap u^0
        KFBI_TRY(lin4<double>(d, ng, s->A, 2.0 * k, u0, -k, um1, c1, lap0, 1.0, lapm1));
        KFBI_TRY(lin4<double>(d, Nb, s->Ag, 2.0 * k, u0g, -k, um1g, c1, lap0g, 1.0, lapm1g));
        KFBI_TRY(lin4<double>(d, ng, s->B, k, u0, -1.0, lap0));
        KFBI_TRY(lin4<double>(d, Nb, s->Bg, k, u0g, -1.0, lap0g));
    } else {
        // Strang: u*^0 = u^0 - i tau/2 lap u^0;  Godunov: the state is u^0
        const cd c = make_cd(0.0, s->p.split == KFBI_SPLIT_GODUNOV ? 0.0 : -0.5 * s->p.tau);
        KFBI_TRY(lin4<cd>(d, ng, s->A, make_cd(1.0, 0.0), u0, c, lap0));
        KFBI_TRY(lin4<cd>(d, Nb, s->Ag, make_cd(1.0, 0.0), u0g, c, lap0g));
    }
    KFBI_HIP(hipMemsetAsync(s->phi, 0, Nb * elem_size(d), d->stream));
    s->initialized = true;
    return KFBI_OK;
}

// One implicit solve of a step.  Returns the trace of u^{n+1} on Gamma that
// the recurrence carries there: g itself for the Dirichlet problem, the
// extracted U+ for the Neumann problem (g is then du/dn).
static int step_solve(kfbi_stepper *s, const void *g_next, void *u_out, const kfbi_solve_opts *opts,
                      kfbi_solve_stats *stats, const void **trace, const GridUpdate *up = nullptr) {
    const bool neu = s->p.bc == KFBI_BC_NEUMANN;
    *trace = neu ? s->tr : g_next;
    return helmholtz_solve(s->dom, s->kre, s->kim, s->f, s->fg, g_next, u_out, s->phi, opts, stats, neu ? 1 : 0,
                           neu ? s->tr : nullptr, up);
}

int kfbi_step_heat(kfbi_stepper *s, const void *g_next, const void *src, const void *srcg, void *u_out,
                   const kfbi_solve_opts *opts, kfbi_solve_stats *stats) {
    if (!s || !g_next || !u_out) { set_error("null argument"); return KFBI_EINVAL; }
    if (s->eq != KFBI_HEAT || !s->initialized) { set_error("not an initialised heat stepper"); return KFBI_EINVAL; }
    kfbi_domain *d = s->dom;
    const int ng = (d->M + 1) * (d->M + 1), Nb = d->Nb;
    KFBI_TRY(lin4_pair<double>(d, ng, Nb, lset<double>(s->f, s->A, src), lset<double>(s->fg, s->Ag, srcg), -1.0,
                               -1.0));
    const void *tr = nullptr;
    int st = step_solve(s, g_next, u_out, opts, stats, &tr);
    if (st != KFBI_OK && st != KFBI_ENOCONV) return st;
    KFBI_TRY(lin4_pair<double>(d, ng, Nb, lset<double>(s->A, u_out, s->f), lset<double>(s->Ag, tr, s->fg),
                               2.0 * s->kre, 1.0));
    return st;
}

int kfbi_step_wave(kfbi_stepper *s, const void *g_next, void *u_out, const kfbi_solve_opts *opts,
                   kfbi_solve_stats *stats) {
    if (!s || !g_next || !u_out) { set_error("null argument"); return KFBI_EINVAL; }
    if (s->eq != KFBI_WAVE || !s->initialized) { set_error("not an initialised wave stepper"); return KFBI_EINVAL; }
    kfbi_domain *d = s->dom;
    const int ng = (d->M + 1) * (d->M + 1), Nb = d->Nb;
    KFBI_TRY(lin4_pair<double>(d, ng, Nb, lset<double>(s->f, s->A), lset<double>(s->fg, s->Ag), -1.0));
    const void *tr = nullptr;
    int st = step_solve(s, g_next, u_out, opts, stats, &tr);
    if (st != KFBI_OK && st != KFBI_ENOCONV) return st;
    const double th = s->p.theta, c1 = (1.0 - 2.0 * th) / th, a = s->kre / th;
    // F^{n+2} into the F^n buffer, then swap
    KFBI_TRY(lin4_pair<double>(d, ng, Nb, lset<double>(s->B, u_out, s->A, s->B), lset<double>(s->Bg, tr, s->Ag, s->Bg),
                               a, -c1, -1.0));
    std::swap(s->A, s->B);
    std::swap(s->Ag, s->Bg);
    return st;
}

int kfbi_step_schrodinger(kfbi_stepper *s, const void *g_next, void *u_out, const kfbi_solve_opts *opts,
                          kfbi_solve_stats *stats) {
    if (!s || !g_next || !u_out) { set_error("null argument"); return KFBI_EINVAL; }
    if (s->eq != KFBI_SCHRODINGER || !s->initialized) { set_error("not an initialised Schroedinger stepper"); return KFBI_EINVAL; }
    KFBI_TRY(schr_b_step(s));
    const void *tr = nullptr;
    // Strang splitting with Dirichlet data: the next u* = 2 u^{n+1} - u**
    // (grid and Gamma) is formed by the final solve's inverse transform as it
    // writes u^{n+1}, with the same sums as schr_state_update
    const bool fused = s->p.split != KFBI_SPLIT_GODUNOV && s->p.bc != KFBI_BC_NEUMANN;
    const GridUpdate up{s->A, s->Ag, g_next, 2.0, 0.0, -1.0, 0.0};
    int st = step_solve(s, g_next, u_out, opts, stats, &tr, fused ? &up : nullptr);
    if (st != KFBI_OK && st != KFBI_ENOCONV) return st;
    if (!fused) KFBI_TRY(schr_state_update(s, u_out, tr));
    return st;
}

}  // extern "C"
