// One interface-problem evaluation on the device (Procedure 2 of section
// 3.3; the unified interface problem (3.30) with [u] = phi, [u_n] = 0 and
// F = f~ of eq. 3.25):
//   * jumps of u and its derivatives across Gamma (section 3.2.5),
//   * corrections of the five-point equations at irregular nodes (section
//     3.2.4) -- one thread per irregular node gathers over its own crossed
//     edges, the "decoupled" strategy of section 3.4.2, so no atomics,
//   * the grid solve (gridsolve.hip),
//   * extraction of the interior limit U+ at the collocation points
//     (section 3.2.6) -- one thread per collocation point.
//
// The density phi and its theta-derivatives reach a crossing parameter by
// fourth-order periodic differences at the collocation points and cubic
// Lagrange interpolation in theta; the 3x3 second-derivative system is
// solved in closed form in the (tangent, normal) frame:
//   u_tt = phi_ss - t'.[grad u],  u_tn = t'_x [u_y] - t'_y [u_x],
//   u_nn = f + kappa phi - u_tt,  [Hessian] = Q [[u_tt,u_tn],[u_tn,u_nn]] Q^T,
// Q = (t | n), n = (t_y, -t_x).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kfbi_internal.h"
#include "jumps.h"

namespace kfbi {

namespace {

template <class T>
__global__ __launch_bounds__(128) void k_corrections(CorrArgs<T> A) {
    corrections_body(A, blockIdx.x);
}

// U+(z_k) = sum_p w_p (U(p) + [p outside] J_k(p)); out = g + scale U+
template <class T>
__device__ void extract_body(const ExtArgs<T> &A, int blk) {
    if (A.done && *A.done) return;
    const int k = blk * blockDim.x + threadIdx.x;
    if (k >= A.Nb) return;
    const T *__restrict__ ust = A.ust;
    const int32_t *__restrict__ nid = A.nid;
    extract_point(A, k, [&](int q) { return ust[nid ? nid[6 * k + q] : 6 * k + q]; });
}

template <class T>
__global__ __launch_bounds__(128) void k_extract(ExtArgs<T> A) {
    extract_body(A, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Matrix-vector operators (f = 0).  The corrections and the jump part of the
// extraction are linear in phi and, by the finite-difference and
// interpolation stencils above, each touches a short window of phi: a
// crossed edge reads phi at k0-3 .. k0+4, a collocation point at k-2 .. k+2.
// Their coefficients are obtained once per kappa by evaluating the same
// device code on unit windows, so the iteration applies them as small dense
// stencils.
// ---------------------------------------------------------------------------
template <class T>
__device__ inline void window_derivs(const T *win, int L, double i12d, double i12d2, T &p, T &pt, T &ptt) {
    const T m2 = win[L - 2], m1 = win[L - 1], c0 = win[L], p1 = win[L + 1], p2 = win[L + 2];
    p = c0;
    pt = ((m2 - p2) + (p1 - m1) * 8.0) * i12d;
    ptt = ((p1 + m1) * 16.0 - (p2 + m2) - c0 * 30.0) * i12d2;
}

// PSI: the operator of the Neumann density ([u] = 0, [u_n] = window),
// else of the Dirichlet density ([u] = window, [u_n] = 0)
template <class T, bool PSI>
__global__ void k_build_corr_op(int n_irr, const IrrNode *__restrict__ irr, const Edge *__restrict__ edges, int Nb,
                                double dth, double h, T kappa, T *__restrict__ coef, int32_t *__restrict__ base) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_irr) return;
    const double i12d = 1.0 / (12.0 * dth), i12d2 = 1.0 / (12.0 * dth * dth);
    const IrrNode R = irr[q];
    const double scale = -R.sgn / (h * h);
    // layout: base[s * n_irr + q], coef[(s * 8 + o) * n_irr + q] (consecutive
    // nodes adjacent); an unused slot has base 0 and zero coefficients
    for (int s = 0; s < 4; ++s) {
        if (s >= R.nedge) {
            base[s * n_irr + q] = 0;
            for (int o = 0; o < 8; ++o) coef[(size_t)(s * 8 + o) * n_irr + q] = zero<T>();
            continue;
        }
        const Edge &E = edges[R.edge[s]];
        base[s * n_irr + q] = wrapk(E.k0 - 3, Nb);
        const double dd = R.d[s];
        for (int o = 0; o < 8; ++o) {
            T win[8];
            for (int u = 0; u < 8; ++u) win[u] = zero<T>();
            win[o] = from_re_im<T>(1.0, 0.0);
            T p = zero<T>(), pt = zero<T>(), ptt = zero<T>();
            for (int l = 0; l < 4; ++l) {  // Lagrange nodes k0-1 .. k0+2 = window 2 .. 5
                T a, b, c;
                window_derivs(win, 2 + l, i12d, i12d2, a, b, c);
                p += a * E.w[l];
                pt += b * E.w[l];
                ptt += c * E.w[l];
            }
            Jumps<T> J = PSI ? jumps_psi(E.fr, p, pt) : jumps_dirichlet(E.fr, p, pt, ptt, zero<T>(), kappa);
            const T ua = E.axis == 0 ? J.ux : J.uy;
            const T uaa = E.axis == 0 ? J.uxx : J.uyy;
            coef[(size_t)(s * 8 + o) * n_irr + q] = (J.u + ua * dd + uaa * (0.5 * dd * dd)) * scale;
        }
    }
}

// Merged form of the corrections operator: the windows of a node's crossed
// edges lie within a few collocation spacings of each other, so they are
// summed into one window of kCorrWin coefficients starting at mbase[q]
// (layout mcoef[o * n_irr + q]).  A node whose windows span more than
// kCorrWin points raises *overflow (the caller then keeps the per-edge form).
constexpr int kCorrWin = 16;

template <class T>
__global__ void k_merge_corr_op(int n_irr, int Nb, const T *__restrict__ coef, const int32_t *__restrict__ base,
                                const IrrNode *__restrict__ irr, T *__restrict__ mcoef, int32_t *__restrict__ mbase,
                                int *overflow) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_irr) return;
    const int ne = irr[q].nedge;
    const int ref = base[q];
    int rel[4], lo = 0, hi = 0;
    for (int s = 0; s < ne; ++s) {
        int r = base[s * n_irr + q] - ref;     // signed periodic offset in (-Nb/2, Nb/2]
        if (r > Nb / 2) r -= Nb;
        if (r <= -Nb / 2) r += Nb;
        rel[s] = r;
        lo = r < lo ? r : lo;
        hi = r > hi ? r : hi;
    }
    for (int o = 0; o < kCorrWin; ++o) mcoef[(size_t)o * n_irr + q] = zero<T>();
    mbase[q] = wrapk(ref + lo, Nb);
    if (hi - lo + 8 > kCorrWin) {
        atomicOr(overflow, 1);
        return;
    }
    for (int s = 0; s < ne; ++s)
        for (int o = 0; o < 8; ++o) {
            const size_t dst = (size_t)(rel[s] - lo + o) * n_irr + q;
            mcoef[dst] = mcoef[dst] + coef[(size_t)(s * 8 + o) * n_irr + q];
        }
}

// Weights of the interior normal derivative at collocation point k: the
// first-order coefficients of the same six-point Taylor fit as the value
// weights, n . (U_x, U_y) with n = (t_y, -t_x).  In the 1/h-scaled system of
// the stencil set-up they solve A^T w = (0, n_x/h, n_y/h, 0, 0, 0).
__device__ inline void normal_weights(const Stencil &S, const Frame &fr, double h, double *w) {
    double A[6][7];
    for (int p = 0; p < 6; ++p) {
        const double u = S.xi[p] / h, v = S.eta[p] / h;
        const double row[6] = {1.0, u, v, 0.5 * u * u, u * v, 0.5 * v * v};
        for (int q = 0; q < 6; ++q) A[q][p] = row[q];
    }
    for (int q = 0; q < 6; ++q) A[q][6] = 0.0;
    A[1][6] = fr.ty / h;
    A[2][6] = -fr.tx / h;
    for (int c = 0; c < 6; ++c) {
        int piv = c;
        for (int r = c + 1; r < 6; ++r)
            if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
        if (piv != c)
            for (int q = 0; q < 7; ++q) {
                const double t = A[c][q];
                A[c][q] = A[piv][q];
                A[piv][q] = t;
            }
        const double inv = 1.0 / A[c][c];
        for (int r = c + 1; r < 6; ++r) {
            const double f = A[r][c] * inv;
            for (int q = c; q < 7; ++q) A[r][q] -= f * A[c][q];
        }
    }
    for (int r = 5; r >= 0; --r) {
        double s = A[r][6];
        for (int q = r + 1; q < 6; ++q) s -= A[r][q] * w[q];
        w[r] = s / A[r][r];
    }
}

template <class T, bool PSI>
__global__ void k_build_ext_op(int Nb, double dth, double h, const Colloc *__restrict__ col,
                               const Stencil *__restrict__ st, T kappa, T *__restrict__ bop, double *__restrict__ w6) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= Nb) return;
    const double i12d = 1.0 / (12.0 * dth), i12d2 = 1.0 / (12.0 * dth * dth);
    const Stencil &S = st[k];
    double w[6];
    if (PSI) normal_weights(S, col[k].fr, h, w);
    else
        for (int p = 0; p < 6; ++p) w[p] = S.w[p];
    for (int p = 0; p < 6; ++p) w6[k * 6 + p] = w[p];
    for (int o = 0; o < 5; ++o) {
        T win[5];
        for (int u = 0; u < 5; ++u) win[u] = zero<T>();
        win[o] = from_re_im<T>(1.0, 0.0);
        T p, pt, ptt;
        window_derivs(win, 2, i12d, i12d2, p, pt, ptt);
        Jumps<T> J = PSI ? jumps_psi(col[k].fr, p, pt) : jumps_dirichlet(col[k].fr, p, pt, ptt, zero<T>(), kappa);
        T acc = zero<T>();
        for (int q = 0; q < 6; ++q) {
            if ((S.out_mask >> q) & 1) {
                const double xi = S.xi[q], eta = S.eta[q];
                T jq = J.u + J.ux * xi + J.uy * eta + J.uxx * (0.5 * xi * xi) + J.uxy * (xi * eta) +
                       J.uyy * (0.5 * eta * eta);
                acc += jq * w[q];
            }
        }
        bop[k * 5 + o] = acc;
    }
}

// normal-derivative weights alone (the Neumann right-hand side and checks)
__global__ void k_normal_weights(int Nb, double h, const Colloc *__restrict__ col, const Stencil *__restrict__ st,
                                 double *__restrict__ wn) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= Nb) return;
    double w[6];
    normal_weights(st[k], col[k].fr, h, w);
    for (int p = 0; p < 6; ++p) wn[k * 6 + p] = w[p];
}

template <class T> T kappa_of(double kre, double kim);
template <> double kappa_of<double>(double kre, double) { return kre; }
template <> cd kappa_of<cd>(double kre, double kim) { return make_cd(kre, kim); }

template <class T>
CorrArgs<T> corr_args(kfbi_domain *d, double kre, double kim, const void *phi_base, const int *jptr,
                      const void *fg, void *corr, const int *done, const void *psi = nullptr) {
    CorrArgs<T> A;
    A.n_irr = d->n_irr;
    A.Nb = d->Nb;
    A.irr = d->irr;
    A.edges = d->edges;
    A.dth = 6.283185307179586476925286766559 / d->Nb;
    A.h = d->h;
    A.kappa = kappa_of<T>(kre, kim);
    A.phi_base = (const T *)phi_base;
    A.jptr = jptr;
    A.fg = (const T *)fg;
    A.psi = (const T *)psi;
    A.corr = (T *)corr;
    A.done = done;
    return A;
}

template <class T>
ExtArgs<T> ext_args(kfbi_domain *d, double kre, double kim, const void *ust, const void *phi_base, const int *jptr,
                    const void *fg, const void *g, double scale, void *out_base, int out_add, const int *done,
                    const void *psi = nullptr, const double *wn = nullptr) {
    ExtArgs<T> A;
    A.Nb = d->Nb;
    A.out_add = out_add;
    A.dth = 6.283185307179586476925286766559 / d->Nb;
    A.scale = scale;
    A.col = d->col;
    A.st = d->st;
    A.kappa = kappa_of<T>(kre, kim);
    A.ust = (const T *)ust;
    A.nid = nullptr;
    A.phi_base = (const T *)phi_base;
    A.jptr = jptr;
    A.fg = (const T *)fg;
    A.psi = (const T *)psi;
    A.wn = wn;
    A.g = (const T *)g;
    A.out_base = (T *)out_base;
    A.done = done;
    return A;
}

template <class T>
int launch_corr(kfbi_domain *d, double kre, double kim, const void *phi_base, const int *jptr,
                const void *fg, void *corr, const int *done, const void *psi = nullptr) {
    const int ps = prof_begin(d);
    k_corrections<T><<<(d->n_irr + 127) / 128, 128, 0, d->stream>>>(
        corr_args<T>(d, kre, kim, phi_base, jptr, fg, corr, done, psi));
    KFBI_CHECK_LAUNCH();
    prof_end(d, ps, KFBI_K_CORRECTIONS, (double)d->n_irr * (sizeof(IrrNode) + sizeof(T)));
    return KFBI_OK;
}

template <class T>
int launch_extract(kfbi_domain *d, double kre, double kim, const void *ust, const void *phi_base,
                   const int *jptr, const void *fg, const void *g, double scale, void *out_base,
                   int out_add, const int *done, const void *psi = nullptr, const double *wn = nullptr) {
    const int ps = prof_begin(d);
    k_extract<T><<<(d->Nb + 127) / 128, 128, 0, d->stream>>>(
        ext_args<T>(d, kre, kim, ust, phi_base, jptr, fg, g, scale, out_base, out_add, done, psi, wn));
    KFBI_CHECK_LAUNCH();
    prof_end(d, ps, KFBI_K_EXTRACT, (double)d->Nb * (sizeof(Colloc) + sizeof(Stencil) + 8.0 * sizeof(T)));
    return KFBI_OK;
}

}  // namespace

int compute_corrections_ctl(kfbi_domain *d, double kre, double kim, const void *phi_base, const int *jptr,
                            const void *f_gamma, void *corr_out, const int *done) {
    if (d->cplx) return launch_corr<cd>(d, kre, kim, phi_base, jptr, f_gamma, corr_out, done);
    return launch_corr<double>(d, kre, kim, phi_base, jptr, f_gamma, corr_out, done);
}

int compute_corrections(kfbi_domain *d, double kre, double kim, const void *phi, const void *f_gamma,
                        void *corr_out) {
    return compute_corrections_ctl(d, kre, kim, phi, nullptr, f_gamma, corr_out, nullptr);
}

int extract_boundary_ctl(kfbi_domain *d, double kre, double kim, const void *ust, const void *phi_base,
                         const int *jptr, const void *f_gamma, const void *g, double scale, void *out_base,
                         int out_add, const int *done) {
    if (d->cplx)
        return launch_extract<cd>(d, kre, kim, ust, phi_base, jptr, f_gamma, g, scale, out_base, out_add, done);
    return launch_extract<double>(d, kre, kim, ust, phi_base, jptr, f_gamma, g, scale, out_base, out_add, done);
}

int extract_boundary(kfbi_domain *d, double kre, double kim, const void *ust, const void *phi,
                     const void *f_gamma, const void *g_minus, double scale, void *out) {
    return extract_boundary_ctl(d, kre, kim, ust, phi, nullptr, f_gamma, g_minus, scale, out, 0, nullptr);
}

int compute_corrections_psi_ctl(kfbi_domain *d, double kre, double kim, const void *f_gamma, const void *psi,
                                void *corr_out, const int *done) {
    if (d->cplx) return launch_corr<cd>(d, kre, kim, nullptr, nullptr, f_gamma, corr_out, done, psi);
    return launch_corr<double>(d, kre, kim, nullptr, nullptr, f_gamma, corr_out, done, psi);
}

int ensure_normal_weights(kfbi_domain *d) {
    if (d->wn) return KFBI_OK;
    KFBI_TRY(dalloc(d, (void **)&d->wn, (size_t)d->Nb * 6 * sizeof(double)));
    k_normal_weights<<<(d->Nb + 127) / 128, 128, 0, d->stream>>>(d->Nb, d->h, d->col, d->st, d->wn);
    KFBI_CHECK_LAUNCH();
    return KFBI_OK;
}

int extract_boundary_psi_ctl(kfbi_domain *d, double kre, double kim, const void *ust, const void *f_gamma,
                             const void *psi, bool normal, const void *g, double scale, void *out,
                             const int *done) {
    if (normal) KFBI_TRY(ensure_normal_weights(d));
    const double *wn = normal ? d->wn : nullptr;
    if (d->cplx)
        return launch_extract<cd>(d, kre, kim, ust, nullptr, nullptr, f_gamma, g, scale, out, 0, done, psi, wn);
    return launch_extract<double>(d, kre, kim, ust, nullptr, nullptr, f_gamma, g, scale, out, 0, done, psi, wn);
}

size_t operators_bytes_pending(const kfbi_domain *d) {
    if (d->cop_coef) return 0;
    const size_t es = elem_size(d), ni = (size_t)d->n_irr, Nb = (size_t)d->Nb;
    return ni * 32 * es + ni * 4 * sizeof(int32_t) + ni * kCorrWin * es + ni * sizeof(int32_t) + 256 + Nb * 5 * es +
           Nb * 6 * sizeof(double);
}

int ensure_operators(kfbi_domain *d, double kre, double kim, int bc) {
    if (d->op_valid && d->op_kre == kre && d->op_kim == kim && d->op_bc == bc) return KFBI_OK;
    const size_t es = elem_size(d);
    if (!d->cop_coef) {
        KFBI_TRY(dalloc(d, &d->cop_coef, (size_t)d->n_irr * 32 * es));
        KFBI_TRY(dalloc(d, (void **)&d->cop_base, (size_t)d->n_irr * 4 * sizeof(int32_t)));
        KFBI_TRY(dalloc(d, &d->mcoef, (size_t)d->n_irr * kCorrWin * es));
        KFBI_TRY(dalloc(d, (void **)&d->mbase, (size_t)d->n_irr * sizeof(int32_t) + 256));
        KFBI_TRY(dalloc(d, &d->bop, (size_t)d->Nb * 5 * es));
        KFBI_TRY(dalloc(d, (void **)&d->w6, (size_t)d->Nb * 6 * sizeof(double)));
    }
    // overflow flag lives after the merged bases
    int *overflow = reinterpret_cast<int *>(reinterpret_cast<char *>(d->mbase) +
                                            (((size_t)d->n_irr * sizeof(int32_t) + 127) & ~(size_t)127));
    KFBI_HIP(hipMemsetAsync(overflow, 0, sizeof(int), d->stream));
    const double dth = 6.283185307179586476925286766559 / d->Nb;
    const int gi = (d->n_irr + 127) / 128, gk = (d->Nb + 127) / 128;
    if (d->cplx) {
        const cd kc = make_cd(kre, kim);
        if (bc) {
            k_build_corr_op<cd, true><<<gi, 128, 0, d->stream>>>(d->n_irr, d->irr, d->edges, d->Nb, dth, d->h, kc,
                                                                 (cd *)d->cop_coef, d->cop_base);
            KFBI_CHECK_LAUNCH();
            k_build_ext_op<cd, true><<<gk, 128, 0, d->stream>>>(d->Nb, dth, d->h, d->col, d->st, kc, (cd *)d->bop,
                                                                d->w6);
        } else {
            k_build_corr_op<cd, false><<<gi, 128, 0, d->stream>>>(d->n_irr, d->irr, d->edges, d->Nb, dth, d->h, kc,
                                                                  (cd *)d->cop_coef, d->cop_base);
            KFBI_CHECK_LAUNCH();
            k_build_ext_op<cd, false><<<gk, 128, 0, d->stream>>>(d->Nb, dth, d->h, d->col, d->st, kc, (cd *)d->bop,
                                                                 d->w6);
        }
    } else {
        if (bc) {
            k_build_corr_op<double, true><<<gi, 128, 0, d->stream>>>(d->n_irr, d->irr, d->edges, d->Nb, dth, d->h,
                                                                     kre, (double *)d->cop_coef, d->cop_base);
            KFBI_CHECK_LAUNCH();
            k_build_ext_op<double, true><<<gk, 128, 0, d->stream>>>(d->Nb, dth, d->h, d->col, d->st, kre,
                                                                    (double *)d->bop, d->w6);
        } else {
            k_build_corr_op<double, false><<<gi, 128, 0, d->stream>>>(d->n_irr, d->irr, d->edges, d->Nb, dth, d->h,
                                                                      kre, (double *)d->cop_coef, d->cop_base);
            KFBI_CHECK_LAUNCH();
            k_build_ext_op<double, false><<<gk, 128, 0, d->stream>>>(d->Nb, dth, d->h, d->col, d->st, kre,
                                                                     (double *)d->bop, d->w6);
        }
    }
    KFBI_CHECK_LAUNCH();
    if (d->cplx)
        k_merge_corr_op<cd><<<gi, 128, 0, d->stream>>>(d->n_irr, d->Nb, (const cd *)d->cop_coef, d->cop_base, d->irr,
                                                       (cd *)d->mcoef, d->mbase, overflow);
    else
        k_merge_corr_op<double><<<gi, 128, 0, d->stream>>>(d->n_irr, d->Nb, (const double *)d->cop_coef,
                                                           d->cop_base, d->irr, (double *)d->mcoef, d->mbase,
                                                           overflow);
    KFBI_CHECK_LAUNCH();
    int hov = 0;
    KFBI_HIP(hipMemcpyAsync(&hov, overflow, sizeof(int), hipMemcpyDeviceToHost, d->stream));
    KFBI_HIP(hipStreamSynchronize(d->stream));
    d->op_merged = hov == 0;
    d->op_valid = true;
    d->op_kre = kre;
    d->op_kim = kim;
    d->op_bc = bc;
    return KFBI_OK;
}

int interface_solve(kfbi_domain *d, double kre, double kim, const void *f_grid, const void *f_gamma,
                    const void *phi, void *u_grid_out, void *uplus_out, bool reuse_rhat) {
    if (f_grid && !reuse_rhat) KFBI_TRY(dst_rows_dense(d, f_grid, true, d->rhat));
    KFBI_TRY(compute_corrections(d, kre, kim, phi, f_gamma, d->corr));
    KFBI_TRY(ensure_coefficients(d, kre, kim));
    KFBI_TRY(tridiag_solve(d, f_grid ? d->rhat : nullptr, d->corr, d->uhat));
    if (uplus_out) {
        KFBI_TRY(eval_stencil_nodes(d, d->uhat, d->ust));
        KFBI_TRY(extract_boundary(d, kre, kim, d->ust, phi, f_gamma, nullptr, 1.0, uplus_out));
    }
    if (u_grid_out) KFBI_TRY(idst_rows_dense(d, d->uhat, u_grid_out));
    return KFBI_OK;
}

// batched launches (members of one scalar type: real, or complex with
// complex kappa)
namespace {
template <class T>
__global__ __launch_bounds__(128) void kb_corrections(const CorrArgs<T> *__restrict__ A,
                                                      const BlkMap *__restrict__ map) {
    const BlkMap e = map[blockIdx.x];
    corrections_body(A[e.inst], e.local);
}
template <class T>
__global__ __launch_bounds__(128) void kb_extract(const ExtArgs<T> *__restrict__ A,
                                                  const BlkMap *__restrict__ map) {
    const BlkMap e = map[blockIdx.x];
    extract_body(A[e.inst], e.local);
}
}  // namespace

// the exact size for the batch's scalar type (the stride the kernels index with)
size_t batch_args_size_iface(int kind, bool cplx) {
    if (kind == kBaCorr) return cplx ? sizeof(CorrArgs<cd>) : sizeof(CorrArgs<double>);
    if (kind == kBaExt) return cplx ? sizeof(ExtArgs<cd>) : sizeof(ExtArgs<double>);
    return 0;
}

int batch_blocks_iface(const kfbi_domain *d, int kind) {
    if (kind == kBaCorr) return (d->n_irr + 127) / 128;
    if (kind == kBaExt) return (d->Nb + 127) / 128;
    return 0;
}

void batch_fill_corr(kfbi_domain *d, double kre, double kim, const void *phi, const void *fg, void *corr,
                     const int *done, void *dst) {
    if (d->cplx) *(CorrArgs<cd> *)dst = corr_args<cd>(d, kre, kim, phi, nullptr, fg, corr, done);
    else *(CorrArgs<double> *)dst = corr_args<double>(d, kre, 0.0, phi, nullptr, fg, corr, done);
}

void batch_fill_ext(kfbi_domain *d, double kre, double kim, const void *ust, const void *phi, const void *fg,
                    const void *g, double scale, void *out, const int *done, void *dst) {
    // batched stencil values come one per distinct node
    if (d->cplx) {
        ExtArgs<cd> A = ext_args<cd>(d, kre, kim, ust, phi, nullptr, fg, g, scale, out, 0, done);
        A.nid = d->erow_nid;
        *(ExtArgs<cd> *)dst = A;
    } else {
        ExtArgs<double> A = ext_args<double>(d, kre, 0.0, ust, phi, nullptr, fg, g, scale, out, 0, done);
        A.nid = d->erow_nid;
        *(ExtArgs<double> *)dst = A;
    }
}

int batch_launch_iface(int kind, const void *args, const BlkMap *map, int blocks, hipStream_t s, bool cplx) {
    if (blocks <= 0) return KFBI_OK;
    if (kind == kBaCorr && cplx) kb_corrections<cd><<<blocks, 128, 0, s>>>((const CorrArgs<cd> *)args, map);
    else if (kind == kBaCorr) kb_corrections<double><<<blocks, 128, 0, s>>>((const CorrArgs<double> *)args, map);
    else if (kind == kBaExt && cplx) kb_extract<cd><<<blocks, 128, 0, s>>>((const ExtArgs<cd> *)args, map);
    else if (kind == kBaExt) kb_extract<double><<<blocks, 128, 0, s>>>((const ExtArgs<double> *)args, map);
    else {
        set_error("unknown batched kernel");
        return KFBI_EINVAL;
    }
    KFBI_CHECK_LAUNCH();
    return KFBI_OK;
}

}  // namespace kfbi
