// Domain setup on the device (Procedure 1 of the paper's algorithm summary,
// section 3.3, in the parallel form of section 3.4.2): node classification
// with one thread per grid node, ordered compaction of irregular nodes and
// crossed edges, one thread per crossed edge for the intersection, one
// thread per collocation point for its frame and six-point stencil
// (section 3.2.6).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <algorithm>
#include <vector>

#include "kfbi_internal.h"

namespace kfbi {

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

struct CurveParams {
    int kind, lobes;
    double cx, cy, R, a, b, r0, amp;
};

CurveParams curve_of(const kfbi_domain_desc &D) {
    CurveParams c;
    c.kind = D.kind; c.lobes = D.lobes;
    c.cx = D.cx; c.cy = D.cy; c.R = D.R; c.a = D.a; c.b = D.b; c.r0 = D.r0; c.amp = D.amp;
    return c;
}

// Grid coordinate -L + i h and the strict polynomial inside test.  Every
// operation is rounded on its own (no fused multiply-add), so that the
// classification is a fixed function of the double inputs:
//   disk    (dx*dx + dy*dy) - R*R < 0
//   ellipse (b*b)*(dx*dx) + (a*a)*(dy*dy) - (a*a)*(b*b) < 0
//   star    with q = dx*dx + dy*dy and S = Im((dx + i dy)^m) built by
//           repeated complex multiplication, rho < r0 + amp sin(m theta)
//           multiplied through by rho^m:
//             odd m : A = q^((m+1)/2) - amp*S, inside iff A < 0 or
//                     A*A < (r0*r0)*q^m
//             even m: C = r0*q^(m/2) + amp*S, inside iff C > 0 and
//                     q^(m+1) < C*C
//           and the centre counts as inside.
__device__ __noinline__ double grid_coord(double L, double h, int i) {
#pragma clang fp contract(off)
    return -L + (double)i * h;
}

__device__ __noinline__ double powi_rounded(double v, int e) {
#pragma clang fp contract(off)
    double p = 1.0;
    for (int s = 0; s < e; ++s) p = p * v;
    return p;
}

__device__ __noinline__ bool inside_test(const CurveParams c, double x, double y) {
#pragma clang fp contract(off)
    double dx = x - c.cx;
    double dy = y - c.cy;
    if (c.kind == KFBI_CURVE_DISK) {
        double v = (dx * dx + dy * dy) - c.R * c.R;
        return v < 0.0;
    }
    if (c.kind == KFBI_CURVE_ELLIPSE) {
        double v = ((c.b * c.b) * (dx * dx) + (c.a * c.a) * (dy * dy)) - (c.a * c.a) * (c.b * c.b);
        return v < 0.0;
    }
    if (dx == 0.0 && dy == 0.0) return true;
    double q = dx * dx + dy * dy;
    double pr = 1.0, pim = 0.0;
    for (int s = 0; s < c.lobes; ++s) {
        double nr = pr * dx - pim * dy;
        double ni = pr * dy + pim * dx;
        pr = nr;
        pim = ni;
    }
    const int m = c.lobes;
    if (m & 1) {
        double A = powi_rounded(q, (m + 1) / 2) - c.amp * pim;
        return (A < 0.0) || (A * A < (c.r0 * c.r0) * powi_rounded(q, m));
    }
    double C = c.r0 * powi_rounded(q, m / 2) + c.amp * pim;
    return (C > 0.0) && (powi_rounded(q, m + 1) < C * C);
}

// smooth level function whose zero set is Gamma (negative inside)
__device__ double level_fn(const CurveParams c, double x, double y) {
    double dx = x - c.cx, dy = y - c.cy;
    if (c.kind == KFBI_CURVE_DISK) return hypot(dx, dy) - c.R;
    if (c.kind == KFBI_CURVE_ELLIPSE) {
        double u = dx / c.a, v = dy / c.b;
        return u * u + v * v - 1.0;
    }
    double th = atan2(dy, dx);
    return hypot(dx, dy) - (c.r0 + c.amp * sin(c.lobes * th));
}

__device__ double param_of(const CurveParams c, double x, double y) {
    double dx = x - c.cx, dy = y - c.cy;
    double th = (c.kind == KFBI_CURVE_ELLIPSE) ? atan2(c.a * dy, c.b * dx) : atan2(dy, dx);
    return th < 0.0 ? th + kTwoPi : th;
}

// gamma, gamma', gamma'' at theta
__device__ void curve_derivs(const CurveParams c, double th, double g[2], double g1[2], double g2[2]) {
    double cs = cos(th), sn = sin(th);
    if (c.kind == KFBI_CURVE_DISK) {
        g[0] = c.cx + c.R * cs; g[1] = c.cy + c.R * sn;
        g1[0] = -c.R * sn; g1[1] = c.R * cs;
        g2[0] = -c.R * cs; g2[1] = -c.R * sn;
    } else if (c.kind == KFBI_CURVE_ELLIPSE) {
        g[0] = c.cx + c.a * cs; g[1] = c.cy + c.b * sn;
        g1[0] = -c.a * sn; g1[1] = c.b * cs;
        g2[0] = -c.a * cs; g2[1] = -c.b * sn;
    } else {
        double m = c.lobes;
        double smt = sin(m * th), cmt = cos(m * th);
        double r = c.r0 + c.amp * smt;
        double r1 = c.amp * m * cmt;
        double r2 = -c.amp * m * m * smt;
        g[0] = c.cx + r * cs; g[1] = c.cy + r * sn;
        g1[0] = r1 * cs - r * sn; g1[1] = r1 * sn + r * cs;
        g2[0] = r2 * cs - 2.0 * r1 * sn - r * cs;
        g2[1] = r2 * sn + 2.0 * r1 * cs - r * sn;
    }
}

// unit tangent, its arc-length derivative, speed and d speed/d theta
__device__ Frame frame_at(const CurveParams c, double th, double *px, double *py) {
    double g[2], g1[2], g2[2];
    curve_derivs(c, th, g, g1, g2);
    Frame f;
    f.sigma = sqrt(g1[0] * g1[0] + g1[1] * g1[1]);
    f.tx = g1[0] / f.sigma;
    f.ty = g1[1] / f.sigma;
    f.dsigma = (g1[0] * g2[0] + g1[1] * g2[1]) / f.sigma;
    double tg2 = f.tx * g2[0] + f.ty * g2[1];
    double s2 = f.sigma * f.sigma;
    f.dtx = (g2[0] - f.tx * tg2) / s2;
    f.dty = (g2[1] - f.ty * tg2) / s2;
    if (px) *px = g[0];
    if (py) *py = g[1];
    return f;
}

// -------------------------------------------------------------------------
// kernels
// -------------------------------------------------------------------------

// one thread per node: bit 0 = inside; flags err[0] when an inside node
// lies within three nodes of the box boundary
__global__ void k_classify(CurveParams c, double L, double h, int M, uint8_t *flags, int *err) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y;
    if (i > M || j > M) return;
    double x = grid_coord(L, h, i), y = grid_coord(L, h, j);
    bool in = inside_test(c, x, y);
    flags[(size_t)j * (M + 1) + i] = in ? 1 : 0;
    if (in && (i <= 2 || i >= M - 2 || j <= 2 || j >= M - 2)) atomicOr(err, 1);
}

__device__ inline bool cls(const uint8_t *f, int M, int i, int j) { return f[(size_t)j * (M + 1) + i] & 1; }

__device__ inline bool is_irregular(const uint8_t *f, int M, int i, int j) {
    if (i < 1 || j < 1 || i > M - 1 || j > M - 1) return false;
    bool c0 = cls(f, M, i, j);
    return cls(f, M, i + 1, j) != c0 || cls(f, M, i - 1, j) != c0 || cls(f, M, i, j + 1) != c0 ||
           cls(f, M, i, j - 1) != c0;
}

// one 64-lane wavefront per row: counts of irregular nodes and of crossed
// edges owned by the row (x-edges (i,j)-(i+1,j) and y-edges (i,j)-(i,j+1))
__global__ __launch_bounds__(64) void k_count(const uint8_t *flags, int M, int *cnt_irr, int *cnt_edge) {
    int j = blockIdx.x;
    int lane = threadIdx.x;
    int ci = 0, ce = 0;
    for (int i = lane; i <= M; i += 64) {
        ci += is_irregular(flags, M, i, j);
        if (i < M) ce += cls(flags, M, i, j) != cls(flags, M, i + 1, j);
        if (j < M) ce += cls(flags, M, i, j) != cls(flags, M, i, j + 1);
    }
    for (int off = 32; off > 0; off >>= 1) {
        ci += __shfl_xor(ci, off, 64);
        ce += __shfl_xor(ce, off, 64);
    }
    if (lane == 0) {
        cnt_irr[j] = ci;
        cnt_edge[j] = ce;
    }
}

// ordered compaction within a row: ballot + popcount keeps increasing i
__global__ __launch_bounds__(64) void k_fill(uint8_t *flags, int M, const int *off_irr,
                                             const int *off_edge, int32_t *irr_list, Edge *edges,
                                             int32_t *ex_map, int32_t *ey_map) {
    int j = blockIdx.x;
    int lane = threadIdx.x;
    unsigned long long below = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    int oi = off_irr[j], oe = off_edge[j];
    // irregular nodes (and flag bit 1)
    for (int base = 0; base <= M; base += 64) {
        int i = base + lane;
        bool p = (i <= M) && is_irregular(flags, M, i, j);
        unsigned long long mask = __ballot(p);
        if (p) {
            irr_list[oi + __popcll(mask & below)] = j * (M + 1) + i;
            flags[(size_t)j * (M + 1) + i] |= 2;
        }
        oi += __popcll(mask);
    }
    // x-edges of the row, then y-edges starting in the row
    for (int axis = 0; axis < 2; ++axis) {
        if (axis == 1 && j == M) break;
        for (int base = 0; base <= M; base += 64) {
            int i = base + lane;
            bool p = false;
            if (i <= M) {
                if (axis == 0) p = (i < M) && (cls(flags, M, i, j) != cls(flags, M, i + 1, j));
                else p = cls(flags, M, i, j) != cls(flags, M, i, j + 1);
            }
            unsigned long long mask = __ballot(p);
            if (p) {
                int e = oe + __popcll(mask & below);
                int a = j * (M + 1) + i;
                int b = axis == 0 ? a + 1 : a + (M + 1);
                bool ain = cls(flags, M, i, j);
                Edge E = {};
                E.p_in = ain ? a : b;
                E.q_out = ain ? b : a;
                E.axis = axis;
                edges[e] = E;
                if (axis == 0) ex_map[a] = e; else ey_map[a] = e;
            }
            oe += __popcll(mask);
        }
    }
}

// one thread per crossed edge: bisection of the level function bracketed by
// the two nodes' classes, curve parameter, frame and interpolation weights
__global__ void k_cross(CurveParams c, double L, double h, int M, int Nb, int n_edges, Edge *edges) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_edges) return;
    Edge E = edges[e];
    int pi = E.p_in % (M + 1), pj = E.p_in / (M + 1);
    int qi = E.q_out % (M + 1), qj = E.q_out / (M + 1);
    double lox = grid_coord(L, h, pi), loy = grid_coord(L, h, pj);
    double hix = grid_coord(L, h, qi), hiy = grid_coord(L, h, qj);
    for (int it = 0; it < 64; ++it) {
        double mx = 0.5 * (lox + hix), my = 0.5 * (loy + hiy);
        if (level_fn(c, mx, my) < 0.0) { lox = mx; loy = my; }
        else { hix = mx; hiy = my; }
    }
    E.X = 0.5 * (lox + hix);
    E.Y = 0.5 * (loy + hiy);
    E.theta = param_of(c, E.X, E.Y);
    E.fr = frame_at(c, E.theta, nullptr, nullptr);
    double dth = kTwoPi / Nb;
    int k0 = (int)floor(E.theta / dth);
    if (k0 > Nb - 1) k0 = Nb - 1;
    double s = E.theta / dth - k0;
    E.k0 = k0;
    E.w[0] = -s * (s - 1.0) * (s - 2.0) / 6.0;
    E.w[1] = (s + 1.0) * (s - 1.0) * (s - 2.0) / 2.0;
    E.w[2] = -(s + 1.0) * s * (s - 2.0) / 2.0;
    E.w[3] = (s + 1.0) * s * (s - 1.0) / 6.0;
    edges[e] = E;
}

// one thread per irregular node: its crossed edges and offsets
__global__ void k_irr(double L, double h, int M, int n_irr, const int32_t *irr_list,
                      const uint8_t *flags, const Edge *edges, const int32_t *ex_map,
                      const int32_t *ey_map, IrrNode *irr, int32_t *irr_col) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_irr) return;
    int node = irr_list[t];
    int i = node % (M + 1), j = node / (M + 1);
    IrrNode R;
    R.node = node;
    R.nedge = 0;
    R.row_i = i;
    R.pad = 0;
    R.sgn = (flags[node] & 1) ? 1.0 : -1.0;
    for (int s = 0; s < 4; ++s) { R.edge[s] = -1; R.d[s] = 0.0; }
    // right, left, up, down: the edge and the neighbour across it
    const int nbr_i[4] = {i + 1, i - 1, i, i};
    const int nbr_j[4] = {j, j, j + 1, j - 1};
    int emap[4];
    emap[0] = ex_map[node];
    emap[1] = ex_map[node - 1];
    emap[2] = ey_map[node];
    emap[3] = ey_map[node - (M + 1)];
    for (int s = 0; s < 4; ++s) {
        int e = emap[s];
        if (e < 0) continue;
        const Edge &E = edges[e];
        double other = (s < 2) ? grid_coord(L, h, nbr_i[s]) : grid_coord(L, h, nbr_j[s]);
        double Xa = (s < 2) ? E.X : E.Y;
        R.edge[R.nedge] = e;
        R.d[R.nedge] = other - Xa;
        R.nedge++;
    }
    irr[t] = R;
    irr_col[t] = i;
}

// one thread per collocation point: z_k, frame, stencil and its weights
__global__ void k_colloc(CurveParams c, double L, double h, int M, int Nb, const uint8_t *flags,
                         Colloc *col, Stencil *st, int *err) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= Nb) return;
    double th = kTwoPi * (double)k / (double)Nb;
    Colloc C;
    C.fr = frame_at(c, th, &C.x, &C.y);
    col[k] = C;
    int ci = (int)floor((C.x + L) / h + 0.5);
    int cj = (int)floor((C.y + L) / h + 0.5);
    double xc = grid_coord(L, h, ci), yc = grid_coord(L, h, cj);
    int sx = (C.x >= xc) ? 1 : -1, sy = (C.y >= yc) ? 1 : -1;
    const int di[6] = {0, 1, -1, 0, 0, sx};
    const int dj[6] = {0, 0, 0, 1, -1, sy};
    Stencil S;
    S.out_mask = 0;
    S.pad = 0;
    double A[6][7];
    for (int p = 0; p < 6; ++p) {
        int ii = ci + di[p], jj = cj + dj[p];
        if (ii < 1 || jj < 1 || ii > M - 1 || jj > M - 1) { atomicOr(err, 2); ii = 1; jj = 1; }
        S.node[p] = jj * (M + 1) + ii;
        if (!(flags[S.node[p]] & 1)) S.out_mask |= 1 << p;
        S.xi[p] = grid_coord(L, h, ii) - C.x;
        S.eta[p] = grid_coord(L, h, jj) - C.y;
        // scaled Taylor row [1, xi, eta, xi^2/2, xi eta, eta^2/2] / powers of h;
        // transposed so that the solve gives row 0 of the inverse
        double u = S.xi[p] / h, v = S.eta[p] / h;
        double row[6] = {1.0, u, v, 0.5 * u * u, u * v, 0.5 * v * v};
        for (int q = 0; q < 6; ++q) A[q][p] = row[q];
    }
    for (int q = 0; q < 6; ++q) A[q][6] = (q == 0) ? 1.0 : 0.0;
    // Gaussian elimination with partial pivoting on A^T w = e0
    for (int col_ = 0; col_ < 6; ++col_) {
        int piv = col_;
        for (int r = col_ + 1; r < 6; ++r)
            if (fabs(A[r][col_]) > fabs(A[piv][col_])) piv = r;
        if (piv != col_)
            for (int q = 0; q < 7; ++q) { double t = A[col_][q]; A[col_][q] = A[piv][q]; A[piv][q] = t; }
        double inv = 1.0 / A[col_][col_];
        for (int r = col_ + 1; r < 6; ++r) {
            double f = A[r][col_] * inv;
            for (int q = col_; q < 7; ++q) A[r][q] -= f * A[col_][q];
        }
    }
    double w[6];
    for (int r = 5; r >= 0; --r) {
        double s = A[r][6];
        for (int q = r + 1; q < 6; ++q) s -= A[r][q] * w[q];
        w[r] = s / A[r][r];
    }
    for (int p = 0; p < 6; ++p) S.w[p] = w[p];
    st[k] = S;
}

__global__ void k_tables(int M, double *sine, double *twiddle, double *scu) {
    int m = blockIdx.x * blockDim.x + threadIdx.x;
    // a period and its first quarter again (2M + M/2 entries)
    if (m < 2 * M + M / 2) sine[m] = sinpi_sym(m, M);
    if (m < max(1, M / 32)) {  // the same values as the table at 64 m and 64 m + M/2
        scu[2 * m] = sinpi_sym(64 * m, M);
        scu[2 * m + 1] = sinpi_sym(64 * m + M / 2, M);
    }
    if (m < M) {  // exp(-2 pi i m / 2M)
        twiddle[2 * m] = cospi((double)m / (double)M);
        twiddle[2 * m + 1] = -sinpi((double)m / (double)M);
    }
}

// Temporary device buffers of the set-up, freed on every return path (the
// frees wait for the work queued on them).
struct SetupTemps {
    std::vector<void *> p;
    int alloc(void **out, size_t bytes) {
        const hipError_t e = hipMalloc(out, bytes);
        if (e != hipSuccess) {
            set_error(std::string("hipMalloc: ") + hipGetErrorString(e));
            *out = nullptr;
            return KFBI_ENOMEM;
        }
        p.push_back(*out);
        return KFBI_OK;
    }
    ~SetupTemps() {
        for (void *q : p) (void)hipFree(q);
    }
};

}  // namespace

int build_domain(kfbi_domain *d) {
    const int M = d->M, Nb = d->Nb;
    const double L = d->L, h = d->h;
    CurveParams c = curve_of(d->desc);
    hipStream_t s = d->stream;
    const size_t nodes = (size_t)(M + 1) * (M + 1);

    // the interface must stay at least 3h inside the box (sampled on the host)
    {
        double lim = L - 3.0 * h;
        for (int q = 0; q < 4096; ++q) {
            double th = kTwoPi * q / 4096.0, x, y;
            double cs = cos(th), sn = sin(th);
            if (c.kind == KFBI_CURVE_DISK) { x = c.cx + c.R * cs; y = c.cy + c.R * sn; }
            else if (c.kind == KFBI_CURVE_ELLIPSE) { x = c.cx + c.a * cs; y = c.cy + c.b * sn; }
            else { double r = c.r0 + c.amp * sin(c.lobes * th); x = c.cx + r * cs; y = c.cy + r * sn; }
            if (fabs(x) > lim || fabs(y) > lim) {
                set_error("interface comes within 3h of the box boundary");
                return KFBI_EDOMAIN;
            }
        }
    }

    KFBI_TRY(dalloc(d, (void **)&d->flags, nodes));
    SetupTemps tmp;
    int *err = nullptr, *cnt = nullptr;
    int32_t *ex_map = nullptr, *ey_map = nullptr, *irr_list = nullptr;
    KFBI_TRY(tmp.alloc((void **)&err, 2 * sizeof(int)));
    KFBI_TRY(tmp.alloc((void **)&cnt, 4 * (M + 1) * sizeof(int)));
    KFBI_HIP(hipMemsetAsync(err, 0, 2 * sizeof(int), s));
    KFBI_HIP(hipMemsetAsync(d->flags, 0, nodes, s));

    dim3 gc((M + 1 + 255) / 256, M + 1);
    k_classify<<<gc, 256, 0, s>>>(c, L, h, M, d->flags, err);
    KFBI_CHECK_LAUNCH();
    k_count<<<M + 1, 64, 0, s>>>(d->flags, M, cnt, cnt + (M + 1));
    KFBI_CHECK_LAUNCH();

    std::vector<int> hc(2 * (M + 1));
    int herr = 0;
    KFBI_HIP(hipMemcpyAsync(hc.data(), cnt, 2 * (M + 1) * sizeof(int), hipMemcpyDeviceToHost, s));
    KFBI_HIP(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s));
    KFBI_HIP(hipStreamSynchronize(s));
    if (herr) {
        set_error("an inside node lies within 3h of the box boundary");
        return KFBI_EDOMAIN;
    }
    std::vector<int> off(2 * (M + 1));
    int ti = 0, te = 0;
    for (int j = 0; j <= M; ++j) {
        off[j] = ti; ti += hc[j];
        off[(M + 1) + j] = te; te += hc[(M + 1) + j];
    }
    d->n_irr = ti;
    d->n_edges = te;
    if (ti == 0 || te == 0) {
        set_error("the interface crosses no grid line");
        return KFBI_EDOMAIN;
    }
    // irregular nodes of interior row t (grid row j = t + 1)
    std::vector<int32_t> rowptr(d->n + 1);
    for (int t = 0; t <= d->n; ++t) rowptr[t] = off[t + 1];
    // rows with irregular nodes, heaviest first: the sparse right-hand side
    // of the grid solve is built one row per thread, so neighbouring threads
    // get rows of similar length
    std::vector<int32_t> order;
    for (int t = 0; t < d->n; ++t)
        if (rowptr[t + 1] > rowptr[t]) order.push_back(t);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return rowptr[a + 1] - rowptr[a] > rowptr[b + 1] - rowptr[b];
    });
    d->n_act_rows = (int)order.size();
    // segments in row_order; the segments of one row are consecutive and
    // a segment's last node is the one before the next segment's first,
    // except at the row's end (given by the row pointers)
    std::vector<int32_t> seg_q0, seg_row, row_seg;
    for (int32_t t : order) {
        row_seg.push_back((int32_t)seg_q0.size());
        for (int q = rowptr[t]; q < rowptr[t + 1]; q += kSegLen) {
            seg_q0.push_back(q);
            seg_row.push_back(t);
        }
    }
    row_seg.push_back((int32_t)seg_q0.size());
    d->n_seg = (int)seg_q0.size();
    KFBI_HIP(hipMemcpyAsync(cnt + 2 * (M + 1), off.data(), 2 * (M + 1) * sizeof(int), hipMemcpyHostToDevice, s));

    KFBI_TRY(dalloc(d, (void **)&d->edges, (size_t)te * sizeof(Edge)));
    KFBI_TRY(dalloc(d, (void **)&d->irr, (size_t)ti * sizeof(IrrNode)));
    KFBI_TRY(dalloc(d, (void **)&d->irr_row_ptr, (size_t)(d->n + 1) * sizeof(int32_t)));
    KFBI_TRY(dalloc(d, (void **)&d->irr_col, (size_t)ti * sizeof(int32_t)));
    KFBI_TRY(dalloc(d, (void **)&d->row_order, order.size() * sizeof(int32_t)));
    KFBI_HIP(hipMemcpyAsync(d->row_order, order.data(), order.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    KFBI_TRY(dalloc(d, (void **)&d->seg_q0, seg_q0.size() * sizeof(int32_t)));
    KFBI_HIP(hipMemcpyAsync(d->seg_q0, seg_q0.data(), seg_q0.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    KFBI_TRY(dalloc(d, (void **)&d->seg_row, seg_row.size() * sizeof(int32_t)));
    KFBI_HIP(hipMemcpyAsync(d->seg_row, seg_row.data(), seg_row.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    KFBI_TRY(dalloc(d, (void **)&d->row_seg, row_seg.size() * sizeof(int32_t)));
    KFBI_HIP(hipMemcpyAsync(d->row_seg, row_seg.data(), row_seg.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    {
        std::vector<int32_t> sd(4 * seg_q0.size()), rd(4 * order.size());
        for (size_t g = 0; g < seg_q0.size(); ++g) {
            const int32_t t = seg_row[g], q0 = seg_q0[g];
            sd[4 * g] = q0;
            sd[4 * g + 1] = std::min(q0 + kSegLen, rowptr[t + 1]);
            sd[4 * g + 2] = t;
            sd[4 * g + 3] = 0;
        }
        for (size_t a = 0; a < order.size(); ++a) {
            rd[4 * a] = order[a];
            rd[4 * a + 1] = row_seg[a];
            rd[4 * a + 2] = row_seg[a + 1];
            rd[4 * a + 3] = 0;
        }
        KFBI_TRY(dalloc(d, (void **)&d->seg_desc, sd.size() * sizeof(int32_t)));
        KFBI_HIP(hipMemcpyAsync(d->seg_desc, sd.data(), sd.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        KFBI_TRY(dalloc(d, (void **)&d->row_desc, rd.size() * sizeof(int32_t)));
        KFBI_HIP(hipMemcpyAsync(d->row_desc, rd.data(), rd.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        // segment span of every interior row, padded with empty spans to 64 c rows
        int c64 = 1;
        while (64 * c64 < d->n) c64 <<= 1;
        std::vector<int32_t> rs(2 * (size_t)std::max(64 * c64, d->n), 0);
        for (size_t a = 0; a < order.size(); ++a) {
            rs[2 * (size_t)order[a]] = row_seg[a];
            rs[2 * (size_t)order[a] + 1] = row_seg[a + 1];
        }
        KFBI_TRY(dalloc(d, (void **)&d->row_span, rs.size() * sizeof(int32_t)));
        KFBI_HIP(hipMemcpyAsync(d->row_span, rs.data(), rs.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        KFBI_HIP(hipStreamSynchronize(s));
    }
    KFBI_TRY(tmp.alloc((void **)&ex_map, nodes * sizeof(int32_t)));
    KFBI_TRY(tmp.alloc((void **)&ey_map, nodes * sizeof(int32_t)));
    KFBI_TRY(tmp.alloc((void **)&irr_list, (size_t)ti * sizeof(int32_t)));
    KFBI_HIP(hipMemsetAsync(ex_map, 0xff, nodes * sizeof(int32_t), s));
    KFBI_HIP(hipMemsetAsync(ey_map, 0xff, nodes * sizeof(int32_t), s));
    KFBI_HIP(hipMemcpyAsync(d->irr_row_ptr, rowptr.data(), rowptr.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice, s));

    k_fill<<<M + 1, 64, 0, s>>>(d->flags, M, cnt + 2 * (M + 1), cnt + 3 * (M + 1), irr_list, d->edges,
                                ex_map, ey_map);
    KFBI_CHECK_LAUNCH();
    k_cross<<<(te + 127) / 128, 128, 0, s>>>(c, L, h, M, Nb, te, d->edges);
    KFBI_CHECK_LAUNCH();
    k_irr<<<(ti + 127) / 128, 128, 0, s>>>(L, h, M, ti, irr_list, d->flags, d->edges, ex_map, ey_map, d->irr, d->irr_col);
    KFBI_CHECK_LAUNCH();

    KFBI_TRY(dalloc(d, (void **)&d->col, (size_t)Nb * sizeof(Colloc)));
    KFBI_TRY(dalloc(d, (void **)&d->st, (size_t)Nb * sizeof(Stencil)));
    k_colloc<<<(Nb + 127) / 128, 128, 0, s>>>(c, L, h, M, Nb, d->flags, d->col, d->st, err + 1);
    KFBI_CHECK_LAUNCH();

    KFBI_TRY(dalloc(d, (void **)&d->sine, (2 * (size_t)M + M / 2) * sizeof(double)));
    KFBI_TRY(dalloc(d, (void **)&d->scu, 2 * (size_t)std::max(1, M / 32) * sizeof(double)));
    KFBI_TRY(dalloc(d, (void **)&d->twiddle, 2 * (size_t)M * sizeof(double)));
    k_tables<<<(2 * M + M / 2 + 255) / 256, 256, 0, s>>>(M, d->sine, d->twiddle, d->scu);
    KFBI_CHECK_LAUNCH();

    // inside-node count (host, from the flags; setup only)
    std::vector<uint8_t> hf(nodes);
    KFBI_HIP(hipMemcpyAsync(hf.data(), d->flags, nodes, hipMemcpyDeviceToHost, s));
    KFBI_HIP(hipMemcpyAsync(&herr, err + 1, sizeof(int), hipMemcpyDeviceToHost, s));
    KFBI_HIP(hipStreamSynchronize(s));
    int nin = 0;
    for (size_t q = 0; q < nodes; ++q) nin += hf[q] & 1;
    d->n_inside = nin;
    if (herr) {
        set_error("an extraction stencil reaches the box boundary");
        return KFBI_EDOMAIN;
    }
    // the stencil nodes grouped by grid row: for each interior row holding
    // stencil nodes, the entries (index 6k+p into the stencil values, column)
    std::vector<Stencil> hst(Nb);
    KFBI_HIP(hipMemcpyAsync(hst.data(), d->st, (size_t)Nb * sizeof(Stencil), hipMemcpyDeviceToHost, s));
    KFBI_HIP(hipStreamSynchronize(s));
    std::vector<std::vector<std::pair<int32_t, int32_t>>> per_row(d->n);
    for (int k = 0; k < Nb; ++k)
        for (int p = 0; p < 6; ++p) {
            const int node = hst[k].node[p];
            const int t = node / (M + 1) - 1, i = node % (M + 1);
            per_row[t].push_back({6 * k + p, i});
        }
    std::vector<int32_t> erow_t, erow_ptr, erow_col, erow_nid((size_t)6 * Nb, -1);
    for (int t = 0; t < d->n; ++t) {
        if (per_row[t].empty()) continue;
        auto &pr = per_row[t];
        std::stable_sort(pr.begin(), pr.end(),
                         [](const std::pair<int32_t, int32_t> &a, const std::pair<int32_t, int32_t> &b) {
                             return a.second < b.second;
                         });
        erow_t.push_back(t);
        erow_ptr.push_back((int32_t)erow_col.size());
        for (size_t q = 0; q < pr.size(); ++q) {
            if (q == 0 || pr[q].second != pr[q - 1].second) erow_col.push_back(pr[q].second);
            erow_nid[pr[q].first] = (int32_t)erow_col.size() - 1;
        }
    }
    erow_ptr.push_back((int32_t)erow_col.size());
    d->n_erows = (int)erow_t.size();
    d->n_enodes = (int)erow_col.size();
    for (size_t r = 0; r < erow_t.size(); r += kErowRows) {
        const size_t r1 = std::min(erow_t.size(), r + kErowRows);
        d->erow_blk_max = std::max(d->erow_blk_max, erow_ptr[r1] - erow_ptr[r]);
    }
    d->erow_lo = erow_t.front();
    d->erow_hi = erow_t.back();
    KFBI_TRY(dalloc(d, (void **)&d->erow_t, erow_t.size() * sizeof(int32_t)));
    KFBI_TRY(dalloc(d, (void **)&d->erow_ptr, erow_ptr.size() * sizeof(int32_t)));
    KFBI_TRY(dalloc(d, (void **)&d->erow_col, erow_col.size() * sizeof(int32_t)));
    KFBI_TRY(dalloc(d, (void **)&d->erow_nid, erow_nid.size() * sizeof(int32_t)));
    KFBI_HIP(hipMemcpyAsync(d->erow_nid, erow_nid.data(), erow_nid.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                            s));
    KFBI_HIP(hipMemcpyAsync(d->erow_t, erow_t.data(), erow_t.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    KFBI_HIP(hipMemcpyAsync(d->erow_ptr, erow_ptr.data(), erow_ptr.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                            s));
    KFBI_HIP(hipMemcpyAsync(d->erow_col, erow_col.data(), erow_col.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                            s));
    KFBI_HIP(hipStreamSynchronize(s));
    return KFBI_OK;
}

}  // namespace kfbi
