// Internal declarations of the KFBI HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <string>
#include <vector>

#include "kfbi.h"

namespace kfbi {

// irregular nodes per segment of the sparse right-hand side build
constexpr int kSegLen = 8;

// ---------------------------------------------------------------------------
// scalar types: real double, and an interleaved complex double that matches
// torch's complex128 layout.
// ---------------------------------------------------------------------------
struct cd {
    double x, y;
};

__host__ __device__ inline cd make_cd(double a, double b) { cd r; r.x = a; r.y = b; return r; }
__host__ __device__ inline cd operator+(cd a, cd b) { return make_cd(a.x + b.x, a.y + b.y); }
__host__ __device__ inline cd operator-(cd a, cd b) { return make_cd(a.x - b.x, a.y - b.y); }
__host__ __device__ inline cd operator-(cd a) { return make_cd(-a.x, -a.y); }
__host__ __device__ inline cd operator*(cd a, cd b) { return make_cd(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__host__ __device__ inline cd operator*(double s, cd a) { return make_cd(s * a.x, s * a.y); }
__host__ __device__ inline cd operator*(cd a, double s) { return make_cd(s * a.x, s * a.y); }
__host__ __device__ inline cd operator/(cd a, cd b) {
    // Smith's algorithm
    if (fabs(b.x) >= fabs(b.y)) {
        double r = b.y / b.x, den = b.x + b.y * r;
        return make_cd((a.x + a.y * r) / den, (a.y - a.x * r) / den);
    }
    double r = b.x / b.y, den = b.x * r + b.y;
    return make_cd((a.x * r + a.y) / den, (a.y * r - a.x) / den);
}
__host__ __device__ inline cd &operator+=(cd &a, cd b) { a.x += b.x; a.y += b.y; return a; }
__host__ __device__ inline cd &operator-=(cd &a, cd b) { a.x -= b.x; a.y -= b.y; return a; }

// single-precision counterparts for the mixed-precision grid solve
struct cf {
    float x, y;
};
__host__ __device__ inline cf make_cf(float a, float b) { cf r; r.x = a; r.y = b; return r; }
__host__ __device__ inline cf operator+(cf a, cf b) { return make_cf(a.x + b.x, a.y + b.y); }
__host__ __device__ inline cf operator-(cf a, cf b) { return make_cf(a.x - b.x, a.y - b.y); }
__host__ __device__ inline cf operator*(cf a, cf b) { return make_cf(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__host__ __device__ inline cf operator*(float s, cf a) { return make_cf(s * a.x, s * a.y); }
__host__ __device__ inline cf operator*(cf a, float s) { return make_cf(s * a.x, s * a.y); }
__host__ __device__ inline cf operator*(cf a, double s) { return make_cf((float)s * a.x, (float)s * a.y); }
__host__ __device__ inline cf &operator+=(cf &a, cf b) { a.x += b.x; a.y += b.y; return a; }
__host__ __device__ inline cf &operator-=(cf &a, cf b) { a.x -= b.x; a.y -= b.y; return a; }

// a * b + c and a * b with every fused step written out (nothing left for
// the compiler to contract), so that each kernel inlining them rounds alike
// whatever surrounds it (the tridiagonal sweeps, the extraction sums).  The complex forms take the real part
// as fma(ar, br, fma(-ai, bi, cr)) and the imaginary part as
// fma(ar, bi, fma(ai, br, ci)).
__device__ __forceinline__ double mad_(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float mad_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ cd mad_(cd a, cd b, cd c) {
    return make_cd(__builtin_fma(a.x, b.x, __builtin_fma(-a.y, b.y, c.x)),
                   __builtin_fma(a.x, b.y, __builtin_fma(a.y, b.x, c.y)));
}
__device__ __forceinline__ cf mad_(cf a, cf b, cf c) {
    return make_cf(__builtin_fmaf(a.x, b.x, __builtin_fmaf(-a.y, b.y, c.x)),
                   __builtin_fmaf(a.x, b.y, __builtin_fmaf(a.y, b.x, c.y)));
}
__device__ __forceinline__ cd mad_(cd a, double b, cd c) {
    return make_cd(__builtin_fma(a.x, b, c.x), __builtin_fma(a.y, b, c.y));
}
__device__ __forceinline__ cf mad_(cf a, float b, cf c) {
    return make_cf(__builtin_fmaf(a.x, b, c.x), __builtin_fmaf(a.y, b, c.y));
}
__device__ __forceinline__ double mul_(double a, double b) { return a * b; }
__device__ __forceinline__ float mul_(float a, float b) { return a * b; }
__device__ __forceinline__ cd mul_(cd a, cd b) {
    const double p = a.y * b.y, q = a.y * b.x;
    return make_cd(__builtin_fma(a.x, b.x, -p), __builtin_fma(a.x, b.y, q));
}
__device__ __forceinline__ cf mul_(cf a, cf b) {
    const float p = a.y * b.y, q = a.y * b.x;
    return make_cf(__builtin_fmaf(a.x, b.x, -p), __builtin_fmaf(a.x, b.y, q));
}

// sin(pi q / M) for any integer q (M a power of two), formed from the first
// quarter period so that the tables built from it are exactly odd about M
// and even about M/2: then a kernel may keep only part of the period and
// fold its lookups without changing a value.
__device__ inline double sinpi_sym(int q, int M) {
    q &= 2 * M - 1;
    const bool neg = q >= M;
    int r = q & (M - 1);
    if (r > (M >> 1)) r = M - r;
    const double v = sinpi((double)r / (double)M);
    return neg ? -v : v;
}

// a lookup of sin(pi idx / M), 0 <= idx < 2M, in a half-period table
// S[r] = sin(pi r / M), 0 <= r < M (built by sinpi_sym)
template <class R>
__device__ __forceinline__ R sin_folded(const R *S, int idx, int M) {
    const R v = S[idx & (M - 1)];
    return idx >= M ? -v : v;
}

// Cross-lane exchanges of the wavefront reductions on the VALU (gfx950),
// not through the LDS unit: the partner of lane l differs from l in bit B,
// and for the row mirrors also in lower bits, which the later levels of a
// reduction cover anyway.
//   B = 5, 4: permlane32 / permlane16 swaps (l ^ 32, l ^ 16);
//   B = 3, 2: row mirror (i -> 15 - i in each row of 16), half-row mirror
//             (i -> 7 - i in each half row);
//   B = 1, 0: quad permutations (l ^ 2, l ^ 1).
template <int B>
__device__ __forceinline__ unsigned xl32(unsigned u) {
    const int lane = threadIdx.x & 63;
    if constexpr (B == 5) {
        const auto r = __builtin_amdgcn_permlane32_swap(u, u, false, false);
        return lane < 32 ? r[1] : r[0];
    } else if constexpr (B == 4) {
        const auto r = __builtin_amdgcn_permlane16_swap(u, u, false, false);
        return (lane & 16) ? r[0] : r[1];
    } else if constexpr (B == 3) {
        return (unsigned)__builtin_amdgcn_update_dpp(0, (int)u, 0x140, 0xf, 0xf, false);
    } else if constexpr (B == 2) {
        return (unsigned)__builtin_amdgcn_update_dpp(0, (int)u, 0x141, 0xf, 0xf, false);
    } else if constexpr (B == 1) {
        return (unsigned)__builtin_amdgcn_update_dpp(0, (int)u, 0x4E, 0xf, 0xf, false);
    } else {
        return (unsigned)__builtin_amdgcn_update_dpp(0, (int)u, 0xB1, 0xf, 0xf, false);
    }
}
template <int B>
__device__ __forceinline__ double xl(double v) {
    return __hiloint2double((int)xl32<B>((unsigned)__double2hiint(v)), (int)xl32<B>((unsigned)__double2loint(v)));
}
template <int B>
__device__ __forceinline__ float xl(float v) {
    return __uint_as_float(xl32<B>(__float_as_uint(v)));
}
template <int B>
__device__ __forceinline__ cd xl(cd v) {
    return make_cd(xl<B>(v.x), xl<B>(v.y));
}
template <int B>
__device__ __forceinline__ cf xl(cf v) {
    return make_cf(xl<B>(v.x), xl<B>(v.y));
}

// sum over the wavefront, in every lane, the same bits in every lane (each
// exchange pairs two lanes that add the same two values; all 64 lanes
// active)
template <class T>
__device__ inline T wave_sum(T v) {
    v += xl<5>(v);
    v += xl<4>(v);
    v += xl<3>(v);
    v += xl<2>(v);
    v += xl<1>(v);
    v += xl<0>(v);
    return v;
}

// element type conversions between the FP64 path and the FP32 grid solve
__host__ __device__ inline float to_low(double a) { return (float)a; }
__host__ __device__ inline cf to_low(cd a) { return make_cf((float)a.x, (float)a.y); }
__host__ __device__ inline double to_high(float a) { return (double)a; }
__host__ __device__ inline cd to_high(cf a) { return make_cd((double)a.x, (double)a.y); }
__host__ __device__ inline double to_high(double a) { return a; }
__host__ __device__ inline cd to_high(cd a) { return a; }
template <class S> struct Conv;
template <> struct Conv<double> { __host__ __device__ static double from(double a) { return a; } };
template <> struct Conv<cd> { __host__ __device__ static cd from(cd a) { return a; } };
template <> struct Conv<float> { __host__ __device__ static float from(double a) { return (float)a; } };
template <> struct Conv<cf> { __host__ __device__ static cf from(cd a) { return to_low(a); } };

// generic helpers over double / cd
__host__ __device__ inline double conjv(double a) { return a; }
__host__ __device__ inline cd conjv(cd a) { return make_cd(a.x, -a.y); }
__host__ __device__ inline double abs2(double a) { return a * a; }
__host__ __device__ inline double abs2(cd a) { return a.x * a.x + a.y * a.y; }
__host__ __device__ inline double realv(double a) { return a; }
__host__ __device__ inline double realv(cd a) { return a.x; }
template <class T> __host__ __device__ inline T zero();
template <> __host__ __device__ inline double zero<double>() { return 0.0; }
template <> __host__ __device__ inline cd zero<cd>() { return make_cd(0.0, 0.0); }
template <> __host__ __device__ inline float zero<float>() { return 0.0f; }
template <> __host__ __device__ inline cf zero<cf>() { return make_cf(0.0f, 0.0f); }
template <class T> __host__ __device__ inline T from_re_im(double re, double im);
template <> __host__ __device__ inline double from_re_im<double>(double re, double) { return re; }
template <> __host__ __device__ inline cd from_re_im<cd>(double re, double im) { return make_cd(re, im); }
template <> __host__ __device__ inline float from_re_im<float>(double re, double) { return (float)re; }
template <> __host__ __device__ inline cf from_re_im<cf>(double re, double im) { return make_cf((float)re, (float)im); }
// the FP64 type an element of either precision is assembled in
template <class S> struct High { typedef S type; };
template <> struct High<float> { typedef double type; };
template <> struct High<cf> { typedef cd type; };

// ---------------------------------------------------------------------------
// error handling
// ---------------------------------------------------------------------------
void set_error(const std::string &msg);

#define KFBI_HIP(call)                                                                 \
    do {                                                                               \
        hipError_t _e = (call);                                                        \
        if (_e != hipSuccess) {                                                        \
            ::kfbi::set_error(std::string(#call) + ": " + hipGetErrorString(_e));       \
            return KFBI_EDEVICE;                                                       \
        }                                                                              \
    } while (0)

#define KFBI_CHECK_LAUNCH()                                                            \
    do {                                                                               \
        hipError_t _e = hipGetLastError();                                             \
        if (_e != hipSuccess) {                                                        \
            ::kfbi::set_error(std::string("kernel launch: ") + hipGetErrorString(_e)); \
            return KFBI_EDEVICE;                                                       \
        }                                                                              \
    } while (0)

#define KFBI_TRY(expr)                     \
    do {                                   \
        int _s = (expr);                   \
        if (_s != KFBI_OK) return _s;      \
    } while (0)

// ---------------------------------------------------------------------------
// geometry of one point on Gamma (curve frame, section 3.2.5)
// ---------------------------------------------------------------------------
struct Frame {
    double sigma, dsigma;   // |gamma'|, d|gamma'|/dtheta
    double tx, ty;          // unit tangent
    double dtx, dty;        // dt/ds
};

// per crossed edge: the data the jump computation and the corrections need
struct Edge {
    double X, Y, theta;     // intersection and its curve parameter
    Frame fr;
    int32_t p_in, q_out;    // linear indices of the inside / outside node
    int32_t axis;           // 0: x-edge, 1: y-edge
    int32_t k0;             // Lagrange base: nodes k0-1 .. k0+2 (mod Nb)
    double w[4];            // cubic Lagrange weights
};

// per irregular node: its crossed edges (up to 4) and the signed offsets of
// the neighbour across each edge from the intersection
struct IrrNode {
    int32_t node;           // linear index
    int32_t nedge;
    int32_t edge[4];
    double d[4];            // (other node)_a - X_a along the edge axis
    double sgn;             // +1 inside, -1 outside
    int32_t row_i;          // x index i of the node
    int32_t pad;
};

struct Colloc {
    double x, y;
    Frame fr;
};

struct Stencil {
    int32_t node[6];        // linear indices
    int32_t out_mask;       // bit p set: node p is outside Omega
    int32_t pad;
    double w[6];            // extraction weights (row 0 of A^{-1})
    double xi[6], eta[6];   // node - z
};

// ---------------------------------------------------------------------------
// the domain: everything Procedure 1 builds, resident on the device
// ---------------------------------------------------------------------------
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

}  // namespace kfbi

struct kfbi_domain {
    kfbi_domain_desc desc;
    int M = 0, Nb = 0, n = 0;           // n = M - 1 interior nodes per axis
    double L = 0, h = 0;
    bool cplx = false;
    hipStream_t stream = nullptr;
    int n_inside = 0, n_irr = 0, n_edges = 0;
    size_t bytes = 0;
    std::vector<void *> allocs;         // every device allocation of the domain

    // device data
    uint8_t *flags = nullptr;           // (M+1)^2
    kfbi::Edge *edges = nullptr;        // n_edges
    kfbi::IrrNode *irr = nullptr;       // n_irr, sorted by linear index
    int32_t *irr_row_ptr = nullptr;     // n+1: irregular nodes of interior row t (j = t+1)
    int32_t *irr_col = nullptr;         // n_irr: x index i of each irregular node
    int32_t *row_order = nullptr;       // n_act_rows: interior rows holding irregular nodes,
                                        // by decreasing node count
    int n_act_rows = 0;
    // the irregular nodes of each such row cut into segments of at most
    // kSegLen consecutive nodes: first node seg_q0[s] and row seg_row[s]
    // (a segment ends after kSegLen nodes or at its row's end) and, per row
    // of row_order, its first segment row_seg[a] (n_act_rows + 1 entries)
    int32_t *seg_q0 = nullptr;
    int32_t *seg_row = nullptr;
    int32_t *row_seg = nullptr;
    // the same tables as descriptors of four int32 each, one load apiece:
    // per segment {first node, end node, row, 0}, per row of row_order
    // {row, first segment, end segment, 0}
    int32_t *seg_desc = nullptr;
    int32_t *row_desc = nullptr;
    // per interior row t, {first segment, end segment} of the row (equal
    // for a row without irregular nodes); zero-padded to 64 * c rows, c the
    // rows per lane of a 64-lane mode group, so a lane may read all of its
    // rows
    int32_t *row_span = nullptr;
    int n_seg = 0;
    // the distinct stencil nodes grouped by interior grid row: rows
    // erow_t[r] hold nodes erow_ptr[r] .. erow_ptr[r+1] (column erow_col[j]);
    // stencil value 6k+p is the value of distinct node erow_nid[6k+p];
    // erow_lo .. erow_hi spans every such row
    int32_t *erow_t = nullptr, *erow_ptr = nullptr, *erow_col = nullptr, *erow_nid = nullptr;
    int n_erows = 0, erow_lo = 0, erow_hi = 0, n_enodes = 0;
    int erow_blk_max = 0;  // most nodes in kErowRows consecutive rows
    kfbi::Colloc *col = nullptr;        // Nb
    kfbi::Stencil *st = nullptr;        // Nb
    double *sine = nullptr;             // 2M + M/2: sin(pi m / M), m mod 2M
    // the sine table at the angles 64 m (sin, cos pairs): a mode sum's
    // uniform step angles, m < max(1, M / 32)
    double *scu = nullptr;
    double *twiddle = nullptr;          // 2M complex: exp(-2 pi i m / 2M), m < M

    // scratch for solves (element type T = double or cd; sized for cd)
    void *rhat = nullptr;               // n*n: DST of the dense right-hand side
    void *uhat = nullptr;               // n*n: mode-space solution
    void *corr = nullptr;               // n_irr: corrections
    void *corr_f = nullptr;             // n_irr: corrections of the b-solve (f alone)
    void *ust = nullptr;                // 6*Nb: grid solution at stencil nodes
    void *tmp_grid = nullptr;           // (M+1)^2
    void *vec = nullptr;                // scratch boundary vectors (8*Nb)

    // launch shape of the tridiagonal kernel: modes per workgroup (0: default)
    // and LDS staging of the sparse input (-1: when it fits, 0: never), set by
    // timing at the first solve (the candidates compute the same values)
    int tri_mb = 0, tri_stage = -1;
    int tri_rows = 0;  // sparse launches: 1 the register-row kernel, 0 the LDS-tile kernel
    bool tri_tuned = false;

    // mixed precision (FP32 / complex64 grid solve), allocated on first use
    void *uhat32 = nullptr;
    void *etab32 = nullptr;
    void *elim32 = nullptr;
    int32_t *tconv32 = nullptr;
    float *sine32 = nullptr, *scu32 = nullptr;
    bool coef32_valid = false;
    double coef32_kre = 0, coef32_kim = 0;

    // matrix-vector operators (per kappa and boundary condition):
    // corrections = sum over the <= 4 crossed edges of each irregular node of
    // an 8-point window of the density starting at cop_base; extraction =
    // sum_p w6[k][p] U(stencil p) + a 5-point window of the density around k
    // with coefficients bop.  op_bc 0: the Dirichlet operator (density [u],
    // value weights); 1: the Neumann operator (density [u_n], normal-
    // derivative weights)
    bool op_valid = false;
    double op_kre = 0, op_kim = 0;
    int op_bc = 0;
    double *wn = nullptr;               // Nb * 6 normal-derivative weights
    void *cop_coef = nullptr;           // n_irr * 4 * 8
    int32_t *cop_base = nullptr;        // n_irr * 4 (-1: unused slot)
    void *bop = nullptr;                // Nb * 5
    double *w6 = nullptr;               // Nb * 6
    // merged corrections: one 16-point window per node at mbase (layout
    // mcoef[o * n_irr + q]); op_merged false when some node's windows are
    // too far apart, and the per-edge form is used instead
    void *mcoef = nullptr;
    int32_t *mbase = nullptr;
    bool op_merged = false;

    // tridiagonal coefficient table (per kappa)
    bool coef_valid = false;
    double coef_kre = 0, coef_kim = 0;
    void *etab = nullptr;               // n*n worst case, [t][k]
    void *elim = nullptr;               // n: converged e_inf per mode
    int32_t *tconv = nullptr;           // n: first t that uses the limit

    // GMRES workspace
    void *gm = nullptr;                 // device GmresState (+ basis)
    size_t gm_bytes = 0;
    int last_iters = 0;                 // iterations of the previous solve (chunk sizing)
    int slot_hist[4] = {0, 0, 0, 0};    // grid solves of the last four device-driven solves
                                        // (ring, next entry at slot_pos & 3)
    int slot_pos = 0;
    void *mirror_host = nullptr;        // pinned host copy of the GMRES control block
    void *mirror_dev = nullptr;         //   and its device address
    hipEvent_t ev0 = nullptr, ev1 = nullptr;  // solve timing

    // optional per-kernel timing with HIP events (kfbi_profile_*)
    struct ProfSlot {
        hipEvent_t a, b;
        int kind;
        int tag;                        // -1: always counted; else GMRES chunk position
        double bytes;
    };
    bool prof_on = false;
    int prof_tag = -1;
    std::vector<ProfSlot> prof_live;
    std::vector<hipEvent_t> prof_pool;
    long long prof_count[KFBI_K_COUNT] = {};
    double prof_ms[KFBI_K_COUNT] = {};
    double prof_bytes[KFBI_K_COUNT] = {};
};

namespace kfbi {

// allocation helper: records the pointer in the domain
int dalloc(kfbi_domain *d, void **p, size_t bytes);

// setup (domain.hip)
int build_domain(kfbi_domain *d);
// device address of this device's no-allocation scratch array (noalloc.hip;
// looked up once per device)
int noalloc_scratch(hipStream_t s, void **out);

// grid solve pieces (gridsolve.hip)
int ensure_coefficients(kfbi_domain *d, double kre, double kim);
// R = dense rhs (grid array, nullable) masked to inside nodes when mask_inside
int dst_rows_dense(kfbi_domain *d, const void *grid, bool mask_inside, void *rhat_out);
int dst_rows_dense_corr(kfbi_domain *d, const void *grid, void *rhat_out, double kre, double kim,
                        const void *f_gamma, void *corr_out);
// Uhat = T^{-1} h^2 (rhat (nullable) + synth(corr))
int tridiag_solve(kfbi_domain *d, const void *rhat, const void *corr, void *uhat_out);
int tridiag_solve_ctl(kfbi_domain *d, const void *rhat, const void *corr, void *uhat_out, const int *done);
// U on the full grid from Uhat
int idst_rows_dense(kfbi_domain *d, const void *uhat, void *grid_out);
struct GridUpdate;  // below
int idst_rows_dense_ctl(kfbi_domain *d, const void *uhat, void *grid_out, const int *done,
                        const GridUpdate *up = nullptr);
// U at the 6 Nb stencil nodes
int eval_stencil_nodes(kfbi_domain *d, const void *uhat, void *ust_out);
int eval_extract_boundary(kfbi_domain *d, double kre, double kim, const void *uhat, const void *f_gamma,
                          const void *g, double scale, void *out);
int eval_stencil_nodes_ctl(kfbi_domain *d, const void *uhat, void *ust_out, const int *done, bool low = false);
// K phi at the collocation points from the mode-space solution of phi's
// corrections (merged operator form: stencil weights w6, jump terms bop)
int eval_extract_ctl(kfbi_domain *d, const void *uhat, const void *phi, void *kv_out, const int *done, bool low);
// mixed precision: FP32 / complex64 coefficient tables and grid solve
int ensure_coefficients_low(kfbi_domain *d, double kre, double kim);
int tridiag_solve_low(kfbi_domain *d, const void *corr, void *uhat32_out, const int *done);
// grid solve of the corrections of a density phi (FP64 / complex128, Nb
// values; corrections with the merged operator); low: FP32 / complex64 solve
int tridiag_solve_phi(kfbi_domain *d, const void *phi, void *uhat_out, const int *done, bool low);
// the density of the last solve on the domain (null before the first)
const void *gmres_last_density(kfbi_domain *d);
// corrections of a density with the merged operator (many workgroups),
// plus base (nullable) node by node
int corrections_of_density(kfbi_domain *d, const void *phi, void *corr_out, const int *done,
                           const void *base = nullptr, void *copy_out = nullptr);

// interface pieces (interface.hip)
int compute_corrections(kfbi_domain *d, double kre, double kim, const void *phi,
                        const void *f_gamma, void *corr_out);
int extract_boundary(kfbi_domain *d, double kre, double kim, const void *ust,
                     const void *phi, const void *f_gamma, const void *g_minus,
                     double scale, void *out);
// variants whose density / output slot is base + (*jptr + add) * Nb and that
// return at once when *done is set (device-resident GMRES control)
int compute_corrections_ctl(kfbi_domain *d, double kre, double kim, const void *phi_base,
                            const int *jptr, const void *f_gamma, void *corr_out, const int *done);
int extract_boundary_ctl(kfbi_domain *d, double kre, double kim, const void *ust,
                         const void *phi_base, const int *jptr, const void *f_gamma,
                         const void *g, double scale, void *out_base, int out_add,
                         const int *done);

// build the matrix-vector operators for this kappa (no-op when current)
int ensure_operators(kfbi_domain *d, double kre, double kim, int bc = 0);
// Neumann pieces: corrections with [u] = 0, [u_n] = psi and f (f_gamma
// nullable); extraction with [u_n] = psi (nullable) and f, of the value
// (normal = false) or of the interior normal derivative (normal = true):
// out = g + scale * (extracted), g nullable
int compute_corrections_psi_ctl(kfbi_domain *d, double kre, double kim, const void *f_gamma, const void *psi,
                                void *corr_out, const int *done);
int extract_boundary_psi_ctl(kfbi_domain *d, double kre, double kim, const void *ust, const void *f_gamma,
                             const void *psi, bool normal, const void *g, double scale, void *out,
                             const int *done);
int ensure_normal_weights(kfbi_domain *d);

// one full interface solve IS(f, f_gamma, phi) -> (u grid, U+)
int interface_solve(kfbi_domain *d, double kre, double kim, const void *f_grid,
                    const void *f_gamma, const void *phi, void *u_grid_out,
                    void *uplus_out, bool reuse_rhat);

// GMRES (gmres.hip)
// bc 0: Dirichlet (g_gamma = u on Gamma, density [u]); bc 1: Neumann
// (g_gamma = du/dn, density [u_n]); trace_out (nullable, Neumann) receives
// the interior limit U+ at the collocation points
int helmholtz_solve(kfbi_domain *d, double kre, double kim, const void *f_grid,
                    const void *f_gamma, const void *g_gamma, void *u_grid_out,
                    void *phi_inout, const kfbi_solve_opts *opts, kfbi_solve_stats *stats,
                    int bc = 0, void *trace_out = nullptr, const GridUpdate *up = nullptr);

inline size_t elem_size(const kfbi_domain *d) { return d->cplx ? sizeof(cd) : sizeof(double); }

// ---------------------------------------------------------------------------
// Kernel argument blocks.  Each device kernel body takes one of these and its
// block index; a single-instance launch passes the block by value, a batched
// launch reads one per instance from device memory (see BlkMap).
// ---------------------------------------------------------------------------
// Global-memory view of a pointer held in an argument block.  Batched
// kernels read their argument blocks from device memory, so the compiler
// cannot tell those pointers from LDS ones and would access them with flat
// instructions, whose completion also gates every later LDS wait.  Loads
// and stores through these views are global ones.
template <class T> using gmem = __attribute__((address_space(1))) T;
template <class T> __device__ __forceinline__ const gmem<T> *gview(const T *p) { return (const gmem<T> *)p; }
template <class T> __device__ __forceinline__ gmem<T> *gview(T *p) { return (gmem<T> *)p; }
// Constant-memory view for tables that no kernel writes: a load through it
// at a wavefront-uniform index becomes a scalar load into SGPRs.
template <class T> using cmem = __attribute__((address_space(4))) T;
template <class T> __device__ __forceinline__ const cmem<T> *cview(const T *p) { return (const cmem<T> *)p; }

// element loads and stores through global views (complex elements move as
// one two-lane vector)
typedef double gdv2 __attribute__((ext_vector_type(2)));
typedef float gfv2 __attribute__((ext_vector_type(2)));
template <class T> __device__ __forceinline__ T gld(const gmem<T> *p) {
    if constexpr (std::is_same<T, cd>::value) {
        const gdv2 v = *(const gmem<gdv2> *)p;
        return make_cd(v.x, v.y);
    } else if constexpr (std::is_same<T, cf>::value) {
        const gfv2 v = *(const gmem<gfv2> *)p;
        return make_cf(v.x, v.y);
    } else {
        return *p;
    }
}
template <class T> __device__ __forceinline__ void gst(gmem<T> *p, T v) {
    if constexpr (std::is_same<T, cd>::value) *(gmem<gdv2> *)p = gdv2{v.x, v.y};
    else if constexpr (std::is_same<T, cf>::value) *(gmem<gfv2> *)p = gfv2{v.x, v.y};
    else *p = v;
}

// real scalar type of an element type (sine tables, scale factors)
template <class T> struct Real { typedef double type; };
template <> struct Real<float> { typedef float type; };
template <> struct Real<cf> { typedef float type; };

template <class T>
struct DstArgs {
    int M, logN2;
    const T *in;
    int in_grid;
    const uint8_t *mask;
    T *out;
    int out_grid;
    double scale;
    const double *twiddle;
    const int *done;
    T *upd;         // nullable (grid output only): upd = c0 out + c1 upd, node by node
    T upd_c0, upd_c1;
};

template <class T>
struct ZeroArgs {
    int M;
    T *grid;
    const int *done;
    T *upd;         // nullable: as DstArgs::upd, on the zeroed rows
    T upd_c0, upd_c1;
    const T *upd_g;  // with upd: upd_ag = c0 upd_g + c1 upd_ag on Gamma (nb values)
    T *upd_ag;
    int nb;
};

// An update of a time step's carried state that the final solve's inverse
// transform makes as it writes the grid solution u: a = c0 u + c1 a on the
// grid and ag = c0 g + c1 ag on Gamma (the same sums as the stepper's own
// update kernel; real domains use the real parts)
struct GridUpdate {
    void *a, *ag;
    const void *g;
    double c0r, c0i, c1r, c1i;
};

struct TriSparse {
    const int32_t *irr_col, *row_ptr, *row_order, *seg_q0, *seg_row, *row_seg;
    const int32_t *seg_desc, *row_desc;
    const int32_t *row_span;  // per interior row {first segment, end segment}
    int nnz, n_act, n_seg;
};

template <class T, class TC>
struct TriArgs {
    int M;
    double h2;
    const T *rhat;
    const TC *corr;
    TriSparse sp;
    const typename Real<T>::type *sine;
    const T *etab, *elim;
    const int32_t *tconv;
    T *uhat;
    const int *done;
};

template <class T, class TO>
struct EvalArgs {
    int M, nnodes, node_stride;
    const int32_t *nodes;
    const T *uhat;
    const typename Real<T>::type *sine, *scu;
    TO *out;
    const int *done;
};

template <class TC>
struct CorrPhiArgs {
    const TC *phi;
    int Nb, nnz;
    const TC *mcoef;
    const int32_t *mbase;
    TC *corr;
    const int *done;
    const TC *base;       // nullable: corrections added to the density's
    TC *copy_out;         // nullable: the launch also copies the density here
                          // (workgroups past the corrections' own)
};

template <class T, class TO>
struct EvxArgs {
    int M, Nb, node_stride;
    const int32_t *nodes;
    const T *uhat;
    const typename Real<T>::type *sine, *scu;
    const double *w6;
    const TO *bop;
    const TO *phi;
    TO *kv;
    const int *done;
};

template <class T>
struct CorrArgs {
    int n_irr, Nb;
    const IrrNode *irr;
    const Edge *edges;
    double dth, h;
    T kappa;
    const T *phi_base;
    const int *jptr;
    const T *fg;
    const T *psi;         // nullable: [u_n] = psi (the Neumann density), else 0
    T *corr;
    const int *done;
};

template <class T>
struct ExtArgs {
    int Nb, out_add;
    double dth, scale;
    const Colloc *col;
    const Stencil *st;
    T kappa;
    const T *ust;
    const int32_t *nid;   // null: ust holds the 6 Nb stencil values in order;
                          // else one value per distinct node, 6k+p -> nid[6k+p]
    const T *phi_base;
    const int *jptr;
    const T *fg;
    const T *psi;         // nullable: [u_n] = psi, else 0
    const double *wn;     // nullable: six weights per point replacing the
                          // stencil's own (the normal-derivative weights)
    const T *g;
    T *out_base;
    const int *done;
};

// stencil values by rows: one wavefront per row that holds stencil nodes,
// kErowRows rows per workgroup
constexpr int kErowRows = 8;
constexpr int kErowCols = 1024;  // node columns of a workgroup staged in LDS
template <class T, class TO>
struct ErowArgs {
    int M, n_rows;
    const int32_t *erow_t, *erow_ptr, *erow_col;
    const T *uhat;
    const typename Real<T>::type *sine, *scu;
    TO *ust;
    const int *done;
};

// K phi at the collocation points from the stencil values (merged form)
template <class T>
struct ExmArgs {
    int Nb;
    const T *ust;         // one value per distinct stencil node
    const int32_t *nid;   // stencil value 6k+p -> distinct node
    const double *w6;
    const T *bop;
    const T *phi;
    T *kv;
    const int *done;
};

// batched launches: workgroup b of the launch runs local block `local` of
// instance `inst`
struct BlkMap {
    int inst, local;
};

// ---------------------------------------------------------------------------
// Batched solves (many domains of one scalar type per launch).  Each kernel
// kind has an argument block per member and a block count per member; the
// batch driver lays the members' blocks out in a BlkMap and launches one
// grid.  A kernel indexes the argument blocks with the size of its own
// instantiation, so they are laid out with the exact size for the batch's
// scalar type.
// ---------------------------------------------------------------------------
enum {
    kBaDst = 0,       // DST rows (dense forward or inverse)
    kBaZero,          // first / last grid rows of an output grid
    kBaTri64,         // tridiagonal solve, FP64
    kBaTri32,         // tridiagonal solve, FP32 inner
    kBaEval,          // grid values at the stencil nodes
    kBaEvx64,         // K phi at the collocation points, FP64 grid values
    kBaEvx32,         //   from FP32 grid values
    kBaCorrPhi,       // corrections of a density (merged operator)
    kBaCorr,          // corrections, general form
    kBaExt,           // extraction, general form
    kBaInit,          // GMRES control block init
    kBaSlot,          // GMRES control kernel
    kBaCopy,          // gated copy of the density
    kBaFinal,         // marks a finished member's final solve done
    kBaErow64,        // stencil values by rows, FP64 grid values
    kBaErow32,        //   from FP32 grid values
    kBaExm,           // K phi from stencil values (merged operator)
    kBaKinds
};

struct BatchTriShape {
    int mb, c;
    bool stage;
    bool rows;   // the register-row kernel
    bool dense;  // its dense-input form (the class's dense launches)
    size_t lds, stage_lds;
    int blocks_per;
};

size_t batch_args_size(int kind, bool cplx);
int batch_blocks(const kfbi_domain *d, int kind);
// mb: modes per workgroup (0: each domain's default); stage_pref: -1 stage
// the sparse input when it fits, 0 never, 1 always (error if it does not fit)
// KFBI_TRIDIAG_KERNEL from the environment: 0 "tile", 1 "rows", -1 either
int tri_kernel_pref();
// KFBI_TRIDIAG_KERNEL "tile:<mb>" / "rows:<mb>": the modes per workgroup, 0 when not fixed
int tri_mb_pref();
// KFBI_TRIDIAG_KERNEL "<kernel>:<mb>:<s>": staging of the sparse input, -1 when not fixed
int tri_stage_pref();
// rows: the register-row kernel (64-lane groups of at least 4 rows per lane;
// refused with KFBI_ENOTSUP otherwise); the caller sets dense
int batch_tri_shape(kfbi_domain *const *doms, int n, bool sparse, bool low, BatchTriShape *out, int mb = 0,
                    int stage_pref = -1, bool rows = false);
int batch_tri_blocks(const kfbi_domain *d, int mb);
// cplx: the members are complex (complex128, complex64 inner solves)
int batch_launch(int kind, const void *args, const BlkMap *map, int blocks, int M, const BatchTriShape *shape,
                 hipStream_t s, bool cplx);
void batch_fill_dst(kfbi_domain *d, const void *in, bool in_grid, bool mask_inside, void *out, bool out_grid,
                    double scale, const int *done, void *dst);
void batch_fill_zero(kfbi_domain *d, void *grid, const int *done, void *dst);
void batch_fill_tri(kfbi_domain *d, const void *rhat, const void *corr, void *uhat, const int *done, bool low,
                    void *dst);
void batch_fill_eval(kfbi_domain *d, const void *uhat, void *out, const int *done, void *dst);
void batch_fill_evx(kfbi_domain *d, const void *uhat, const void *phi, void *kv, const int *done, bool low,
                    void *dst);
void batch_fill_corr_phi(kfbi_domain *d, const void *phi, void *corr, const int *done, void *dst,
                         const void *base = nullptr);
void batch_fill_erow(kfbi_domain *d, const void *uhat, void *ust, const int *done, bool low, void *dst);
void batch_fill_exm(kfbi_domain *d, const void *ust, const void *phi, void *kv, const int *done, void *dst);
// interface.hip
size_t batch_args_size_iface(int kind, bool cplx);
int batch_blocks_iface(const kfbi_domain *d, int kind);
void batch_fill_corr(kfbi_domain *d, double kre, double kim, const void *phi, const void *fg, void *corr,
                     const int *done, void *dst);
void batch_fill_ext(kfbi_domain *d, double kre, double kim, const void *ust, const void *phi, const void *fg,
                    const void *g, double scale, void *out, const int *done, void *dst);
int batch_launch_iface(int kind, const void *args, const BlkMap *map, int blocks, hipStream_t s, bool cplx);

// batched Helmholtz solves (gmres.hip)
int batch_create(kfbi_domain *const *doms, int n, kfbi_batch **out);
void batch_destroy(kfbi_batch *b);
// device bytes of the tables a domain allocates on first use, while not yet allocated
size_t operators_bytes_pending(const kfbi_domain *d);
size_t low_tables_bytes_pending(const kfbi_domain *d);
int tune_tridiag(kfbi_domain *d);
int replay_slot(kfbi_domain *d, int reps, double *avg_ms, double *bytes);
int batch_size(const kfbi_batch *b);
kfbi_domain *batch_domain(const kfbi_batch *b, int q);
int batch_tuning(const kfbi_batch *b, int cap, int32_t *rows, double *us, int32_t *n_rows);
// kappa_im (nullable: 0) only for a batch of complex domains
int batch_helmholtz(kfbi_batch *b, const double *kappa, const double *kappa_im, const void *const *f_grid,
                    const void *const *f_gamma, const void *const *g_gamma, void *const *u_out,
                    void *const *phi_inout, const kfbi_solve_opts *opts, kfbi_solve_stats *stats,
                    const uint8_t *active = nullptr);
bool batch_complex(const kfbi_batch *b);

// kernel timing: prof_begin returns a slot (or -1 when profiling is off);
// prof_end closes it with the launch's algorithmic bytes; prof_flush waits
// for the recorded events and accumulates every slot whose tag is -1 or
// below keep_tags_below (GMRES launches that found the solve finished are
// dropped).
int prof_begin(kfbi_domain *d);
void prof_end(kfbi_domain *d, int slot, int kind, double bytes);
int prof_flush(kfbi_domain *d, int keep_tags_below, int keep_tag = -1);

}  // namespace kfbi
