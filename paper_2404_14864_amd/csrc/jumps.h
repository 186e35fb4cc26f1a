// Jump conditions of the interface problem at the boundary (eqs. 3.13-3.16:
// [u], the tangential and normal derivatives from the density and f, the
// second derivatives from the PDE) and the six-point extraction of U+ at a
// collocation point (eq. 3.36), shared by the general correction and
// extraction kernels and the fused launches of the b-solve.
#pragma once

#include "kfbi_internal.h"

namespace kfbi {
namespace {

template <class T> struct Jumps {
    T u, ux, uy, uxx, uxy, uyy;
};

template <class T>
__device__ inline Jumps<T> jumps_dirichlet(const Frame &f, T phi, T pt, T ptt, T fval, T kappa) {
    Jumps<T> J;
    const double inv = 1.0 / f.sigma;
    const T ps = pt * inv;
    const T pss = (ptt - ps * f.dsigma) * (inv * inv);
    J.u = phi;
    J.ux = ps * f.tx;
    J.uy = ps * f.ty;
    const T rtt = pss - (J.ux * f.dtx + J.uy * f.dty);
    const T rtn = J.uy * f.dtx - J.ux * f.dty;
    const T rnn = fval + kappa * phi - rtt;
    const double c = f.tx, s = f.ty;
    J.uxx = rtt * (c * c) + rtn * (2.0 * c * s) + rnn * (s * s);
    J.uxy = rtt * (c * s) + rtn * (s * s - c * c) - rnn * (s * c);
    J.uyy = rtt * (s * s) - rtn * (2.0 * s * c) + rnn * (c * c);
    return J;
}

// The jumps of a density psi = [u_n] alone ([u] = 0, f = 0): the tangential
// derivative of [u] vanishes, so [grad u] = psi n with n = (t_y, -t_x); the
// tangential-normal second derivative picks up psi_s and the curvature terms
// of the same rows as above, and [lap u] = kappa [u] + [f] = 0 gives the
// normal-normal one.
template <class T>
__device__ inline Jumps<T> jumps_psi(const Frame &f, T psi, T pst) {
    Jumps<T> J;
    const T pss = pst * (1.0 / f.sigma);
    J.u = zero<T>();
    J.ux = psi * f.ty;
    J.uy = psi * (-f.tx);
    const T rtt = zero<T>() - (J.ux * f.dtx + J.uy * f.dty);
    const T rtn = pss + J.uy * f.dtx - J.ux * f.dty;
    const T rnn = zero<T>() - rtt;
    const double c = f.tx, s = f.ty;
    J.uxx = rtt * (c * c) + rtn * (2.0 * c * s) + rnn * (s * s);
    J.uxy = rtt * (c * s) + rtn * (s * s - c * c) - rnn * (s * c);
    J.uyy = rtt * (s * s) - rtn * (2.0 * s * c) + rnn * (c * c);
    return J;
}

template <class T>
__device__ inline void add_jumps(Jumps<T> &J, const Jumps<T> &P) {
    J.u += P.u;
    J.ux += P.ux;
    J.uy += P.uy;
    J.uxx += P.uxx;
    J.uxy += P.uxy;
    J.uyy += P.uyy;
}

__device__ inline int wrapk(int k, int Nb) {
    k %= Nb;
    return k < 0 ? k + Nb : k;
}

// phi, phi_theta, phi_thetatheta at collocation point k (periodic 4th-order
// central differences)
template <class T>
__device__ inline void bdata(const T *phi, int Nb, int k, double i12d, double i12d2, T &p, T &pt, T &ptt) {
    T m2 = phi[wrapk(k - 2, Nb)], m1 = phi[wrapk(k - 1, Nb)], c0 = phi[k];
    T p1 = phi[wrapk(k + 1, Nb)], p2 = phi[wrapk(k + 2, Nb)];
    p = c0;
    pt = ((m2 - p2) + (p1 - m1) * 8.0) * i12d;
    ptt = ((p1 + m1) * 16.0 - (p2 + m2) - c0 * 30.0) * i12d2;
}

template <class T>
__device__ inline const T *at_slot(const T *base, const int *jptr, int add, size_t stride) {
    if (!base) return nullptr;
    return base + (jptr ? (size_t)(*jptr + add) * stride : 0);
}


// the correction at each irregular node: the jumps at its edges' crossings
// expanded along the edge (eq. 3.35), one thread per node
template <class T>
__device__ void corrections_body(const CorrArgs<T> &A, int blk) {
    const int n_irr = A.n_irr, Nb = A.Nb;
    const IrrNode *__restrict__ irr = A.irr;
    const Edge *__restrict__ edges = A.edges;
    const double dth = A.dth, h = A.h;
    const T kappa = A.kappa;
    const T *phi_base = A.phi_base;
    const int *jptr = A.jptr;
    const T *__restrict__ fg = A.fg;
    const T *__restrict__ psi = A.psi;
    T *__restrict__ corr = A.corr;
    if (A.done && *A.done) return;
    int q = blk * blockDim.x + threadIdx.x;
    if (q >= n_irr) return;
    const T *phi = at_slot(phi_base, jptr, 0, (size_t)Nb);
    const double i12d = 1.0 / (12.0 * dth), i12d2 = 1.0 / (12.0 * dth * dth);
    const IrrNode R = irr[q];
    T acc = zero<T>();
    for (int s = 0; s < R.nedge; ++s) {
        const Edge &E = edges[R.edge[s]];
        T p = zero<T>(), pt = zero<T>(), ptt = zero<T>(), fv = zero<T>();
        for (int o = 0; o < 4; ++o) {
            int kk = wrapk(E.k0 - 1 + o, Nb);
            double w = E.w[o];
            if (phi) {
                T a, b, c;
                bdata(phi, Nb, kk, i12d, i12d2, a, b, c);
                p += a * w;
                pt += b * w;
                ptt += c * w;
            }
            if (fg) fv += fg[kk] * w;
        }
        Jumps<T> J = jumps_dirichlet(E.fr, p, pt, ptt, fv, kappa);
        if (psi) {
            T s = zero<T>(), st = zero<T>();
            for (int o = 0; o < 4; ++o) {
                T a, b, c;
                bdata(psi, Nb, wrapk(E.k0 - 1 + o, Nb), i12d, i12d2, a, b, c);
                s += a * E.w[o];
                st += b * E.w[o];
            }
            add_jumps(J, jumps_psi(E.fr, s, st));
        }
        const T ua = E.axis == 0 ? J.ux : J.uy;
        const T uaa = E.axis == 0 ? J.uxx : J.uyy;
        const double dd = R.d[s];
        acc += J.u + ua * dd + uaa * (0.5 * dd * dd);
    }
    corr[q] = acc * (-R.sgn / (h * h));
}

// U+(z_k) = sum_p w_p (U(p) + [p outside] J_k(p)) at collocation point k,
// out[k] = g[k] + scale U+; uval(p) gives the grid value at stencil node p
// (from memory, or from LDS where the caller evaluated it)
template <class T, class UV>
__device__ inline void extract_point(const ExtArgs<T> &A, int k, const UV &uval) {
    const int Nb = A.Nb, out_add = A.out_add;
    const double dth = A.dth, scale = A.scale;
    const Colloc *__restrict__ col = A.col;
    const Stencil *__restrict__ st = A.st;
    const T kappa = A.kappa;
    const T *phi_base = A.phi_base;
    const int *jptr = A.jptr;
    const T *__restrict__ fg = A.fg;
    const T *__restrict__ psi = A.psi;
    const double *__restrict__ wn = A.wn;
    const T *__restrict__ g = A.g;
    T *out_base = A.out_base;
    const T *phi = at_slot(phi_base, jptr, 0, (size_t)Nb);
    T *out = out_base + (jptr ? (size_t)(*jptr + out_add) * Nb : 0);
    const double i12d = 1.0 / (12.0 * dth), i12d2 = 1.0 / (12.0 * dth * dth);
    T p = zero<T>(), pt = zero<T>(), ptt = zero<T>();
    if (phi) bdata(phi, Nb, k, i12d, i12d2, p, pt, ptt);
    T fv = fg ? fg[k] : zero<T>();
    Jumps<T> J = jumps_dirichlet(col[k].fr, p, pt, ptt, fv, kappa);
    if (psi) {
        T a, b, c;
        bdata(psi, Nb, k, i12d, i12d2, a, b, c);
        add_jumps(J, jumps_psi(col[k].fr, a, b));
    }
    const Stencil &S = st[k];
    T up = zero<T>();
    for (int q = 0; q < 6; ++q) {
        T val = uval(q);
        if ((S.out_mask >> q) & 1) {
            const double xi = S.xi[q], eta = S.eta[q];
            val += J.u + J.ux * xi + J.uy * eta + J.uxx * (0.5 * xi * xi) + J.uxy * (xi * eta) +
                   J.uyy * (0.5 * eta * eta);
        }
        up += val * (wn ? wn[6 * k + q] : S.w[q]);
    }
    T res = up * scale;
    if (g) res += g[k];
    out[k] = res;
}

}  // namespace
}  // namespace kfbi
