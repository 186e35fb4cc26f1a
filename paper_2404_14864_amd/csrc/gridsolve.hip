// Five-point (Delta_h - kappa) solve on the box with u = 0 on dB (eq. 3.31),
// by a sine transform in x and one tridiagonal solve per x-mode in y.
//
// With R^[t][k] = sum_i R[t][i] sin(pi i k / M) (DST-I along x, modes
// k = 1..M-1) the system decouples into, for every mode k,
//
//     U^_{t-1} - d_k U^_t + U^_{t+1} = h^2 R^_t,   U^_0 = U^_M = 0,
//     d_k = 2 + 4 sin^2(pi k / 2M) + kappa h^2,
//
// which is strictly diagonally dominant (|d_k| > 2, also for complex kappa),
// and U = (2/M) DST-I(U^) row by row.
//
// Layout: mode-space arrays are n x n (n = M - 1), row t (grid row j = t+1)
// major, mode fastest: element (t, k-1) at t*n + (k-1).
//
// Kernels
//   k_dst_rows      dense DST-I of whole rows through a radix-2 FFT of the
//                   odd extension (length 2M) held in LDS; two real rows are
//                   packed into one complex transform.
//   k_coef          Thomas coefficients e_t of every mode (per kappa).
//   k_tridiag       one wavefront per mode: the Thomas forward and backward
//                   recurrences are first-order affine recurrences, solved as
//                   a chunked scan -- each lane composes the affine maps of
//                   its rows, a wavefront-shuffle scan combines the lanes,
//                   and each lane replays its rows.  The right-hand side of a
//                   correction-only solve is sparse (irregular nodes only), so
//                   its x-transform is synthesised in place from a sine table
//                   instead of being read from memory.
//   k_eval_nodes    U at single grid nodes: one wavefront per node reduces
//                   the inverse transform of its row.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include <cstdlib>
#include <cstring>

#include "kfbi_internal.h"
#include "jumps.h"

namespace kfbi {

namespace {

template <class T> struct Shfl;
template <> struct Shfl<double> {
    __device__ static double up(double v, int o, int w = 64) { return __shfl_up(v, o, w); }
    __device__ static double down(double v, int o, int w = 64) { return __shfl_down(v, o, w); }
    __device__ static double xr(double v, int o) { return __shfl_xor(v, o, 64); }
};
template <> struct Shfl<cd> {
    __device__ static cd up(cd v, int o, int w = 64) { return make_cd(__shfl_up(v.x, o, w), __shfl_up(v.y, o, w)); }
    __device__ static cd down(cd v, int o, int w = 64) {
        return make_cd(__shfl_down(v.x, o, w), __shfl_down(v.y, o, w));
    }
    __device__ static cd xr(cd v, int o) { return make_cd(__shfl_xor(v.x, o, 64), __shfl_xor(v.y, o, 64)); }
};

template <> struct Shfl<float> {
    __device__ static float up(float v, int o, int w = 64) { return __shfl_up(v, o, w); }
    __device__ static float down(float v, int o, int w = 64) { return __shfl_down(v, o, w); }
    __device__ static float xr(float v, int o) { return __shfl_xor(v, o, 64); }
};
template <> struct Shfl<cf> {
    __device__ static cf up(cf v, int o, int w = 64) { return make_cf(__shfl_up(v.x, o, w), __shfl_up(v.y, o, w)); }
    __device__ static cf down(cf v, int o, int w = 64) {
        return make_cf(__shfl_down(v.x, o, w), __shfl_down(v.y, o, w));
    }
    __device__ static cf xr(cf v, int o) { return make_cf(__shfl_xor(v.x, o, 64), __shfl_xor(v.y, o, 64)); }
};

template <class T> __device__ inline T one();
template <> __device__ inline double one<double>() { return 1.0; }
template <> __device__ inline cd one<cd>() { return make_cd(1.0, 0.0); }
template <> __device__ inline float one<float>() { return 1.0f; }
template <> __device__ inline cf one<cf>() { return make_cf(1.0f, 0.0f); }


__device__ inline unsigned bitrev(unsigned m, int bits) { return __brev(m) >> (32 - bits); }

// c0 x0 + c1 x1 summed from zero in this order (the stepper's update kernel)
template <class T>
__device__ __forceinline__ T lin2(T c0, T x0, T c1, T x1) {
    T acc = zero<T>();
    acc += c0 * x0;
    acc += c1 * x1;
    return acc;
}


// ---------------------------------------------------------------------------
// dense DST-I of rows.
//   in(t, i)  for i = 1..M-1 at in[in_off(t) + i - 1]
//   out(t, k) for k = 1..M-1 at out[out_off(t) + k - 1], scaled by `scale`
// grid layout: row t at (t+1)*(M+1) + 1;  mode layout: row t at t*n.
// Real rows are paired (t = 2b, 2b+1) into one complex transform
// z = y1 + i y2 of the odd extensions, whose transform is Z_k = 2 S2_k -
// 2i S1_k; a complex row's transform is Y_k = -2i S_k.
// ---------------------------------------------------------------------------
template <class T>
__device__ void dst_rows_body(const DstArgs<T> &A, int blk) {
    const int M = A.M, logN2 = A.logN2;
    const gmem<T> *in = gview(A.in);
    const bool in_grid = A.in_grid, out_grid = A.out_grid;
    const gmem<uint8_t> *mask = gview(A.mask);
    gmem<T> *out = gview(A.out);
    const double scale = A.scale;
    const gmem<double> *twiddle = gview(A.twiddle);
    if (A.done && *gview(A.done)) return;
    extern __shared__ double lds[];
    double2 *a = reinterpret_cast<double2 *>(lds);
    const int n = M - 1, N2 = 2 * M;
    constexpr bool CPLX = sizeof(T) == sizeof(cd);
    const int rows_per = CPLX ? 1 : 2;
    const int t_first = blk * rows_per;
    // load the odd extension, bit-reversed
    for (int m = threadIdx.x; m < N2; m += blockDim.x) {
        double re = 0.0, im = 0.0;
        int i = (m <= M) ? m : N2 - m;      // position in the row
        double sgn = (m <= M) ? 1.0 : -1.0;
        if (i >= 1 && i <= n) {
            for (int r = 0; r < rows_per; ++r) {
                int t = t_first + r;
                if (t >= n) continue;
                size_t idx = in_grid ? (size_t)(t + 1) * (M + 1) + i : (size_t)t * n + (i - 1);
                bool keep = (mask == nullptr) || (mask[(size_t)(t + 1) * (M + 1) + i] & 1);
                if (!keep) continue;
                if constexpr (CPLX) {
                    const cd v = gld(in + idx);
                    re = sgn * v.x;
                    im = sgn * v.y;
                } else {
                    double v = gld(in + idx);
                    if (r == 0) re = sgn * v; else im = sgn * v;
                }
            }
        }
        a[bitrev(m, logN2)] = make_double2(re, im);
    }
    __syncthreads();
    // in-place radix-2 decimation-in-time, twiddle exp(-2 pi i m / N2).
    // Stages are taken three at a time: each thread carries a group of eight
    // points through three stages in registers, so there is one LDS round
    // trip and one barrier per three stages.  The logN2 mod 3 stages left
    // over go first, as a single stage or a pair.
    auto tw = [&](int m, double &wr, double &wi) {
        wr = twiddle[2 * m];
        wi = twiddle[2 * m + 1];
    };
    // butterfly (x, y) <- (x + w y, x - w y)
    auto bfly = [](double2 &x, double2 &y, double wr, double wi) {
        const double vr = y.x * wr - y.y * wi, vi = y.x * wi + y.y * wr;
        y = make_double2(x.x - vr, x.y - vi);
        x = make_double2(x.x + vr, x.y + vi);
    };
    int len = 2, tstep = M;
    const int lead = logN2 % 3;
    if (lead == 1) {
        for (int b = threadIdx.x; b < M; b += blockDim.x) {
            const int i0 = 2 * b, i1 = i0 + 1;
            double wr, wi;
            tw(0, wr, wi);
            double2 u = a[i0], v = a[i1];
            bfly(u, v, wr, wi);
            a[i0] = u;
            a[i1] = v;
        }
        __syncthreads();
        len = 4;
        tstep = M >> 1;
    } else if (lead == 2) {
        // stages of lengths 2 and 4: groups of four points
        for (int b = threadIdx.x; b < (M >> 1); b += blockDim.x) {
            const int i0 = 4 * b;
            double2 x0 = a[i0], x1 = a[i0 + 1], x2 = a[i0 + 2], x3 = a[i0 + 3];
            double wr, wi;
            tw(0, wr, wi);
            bfly(x0, x1, wr, wi);
            bfly(x2, x3, wr, wi);
            bfly(x0, x2, wr, wi);
            tw(M >> 1, wr, wi);
            bfly(x1, x3, wr, wi);
            a[i0] = x0;
            a[i0 + 1] = x1;
            a[i0 + 2] = x2;
            a[i0 + 3] = x3;
        }
        __syncthreads();
        len = 8;
        tstep = M >> 2;
    }
    for (; len <= M; len <<= 3, tstep >>= 3) {
        // stages of lengths len, 2 len, 4 len on the points
        // i0 + q half, q < 8 (i0 = grp 8 half + pos, pos < half)
        const int half = len >> 1, t2 = tstep >> 1, t3 = tstep >> 2;
        for (int b = threadIdx.x; b < (M >> 2); b += blockDim.x) {
            const int grp = b / half, pos = b - grp * half;
            const int i0 = grp * 8 * half + pos;
            double2 x[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) x[q] = a[i0 + q * half];
            double wr, wi;
            tw(pos * tstep, wr, wi);
#pragma unroll
            for (int q = 0; q < 8; q += 2) bfly(x[q], x[q + 1], wr, wi);
            double wr2, wi2;
            tw(pos * t2, wr, wi);
            tw((pos + half) * t2, wr2, wi2);
            bfly(x[0], x[2], wr, wi);
            bfly(x[1], x[3], wr2, wi2);
            bfly(x[4], x[6], wr, wi);
            bfly(x[5], x[7], wr2, wi2);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                tw((pos + q * half) * t3, wr, wi);
                bfly(x[q], x[q + 4], wr, wi);
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) a[i0 + q * half] = x[q];
        }
        __syncthreads();
    }
    // unpack (and, with upd, the state update at each written node)
    T *upd = A.upd;
    for (int k = 1 + threadIdx.x; k <= n; k += blockDim.x) {
        double2 Z = a[k];
        for (int r = 0; r < rows_per; ++r) {
            int t = t_first + r;
            if (t >= n) continue;
            size_t idx = out_grid ? (size_t)(t + 1) * (M + 1) + k : (size_t)t * n + (k - 1);
            T val;
            if constexpr (CPLX) {
                // S_k = i Y_k / 2
                val = make_cd(-0.5 * scale * Z.y, 0.5 * scale * Z.x);
            } else {
                double v = (r == 0) ? -0.5 * Z.y : 0.5 * Z.x;
                val = scale * v;
            }
            gst(out + idx, val);
            if (upd) upd[idx] = lin2(A.upd_c0, val, A.upd_c1, upd[idx]);
        }
    }
    if (out_grid) {  // boundary columns of the interior rows
        for (int r = threadIdx.x; r < rows_per; r += blockDim.x) {
            int t = t_first + r;
            if (t >= n) continue;
            size_t base = (size_t)(t + 1) * (M + 1);
            gst(out + base, zero<T>());
            gst(out + base + M, zero<T>());
            if (upd) {
                upd[base] = lin2(A.upd_c0, zero<T>(), A.upd_c1, upd[base]);
                upd[base + M] = lin2(A.upd_c0, zero<T>(), A.upd_c1, upd[base + M]);
            }
        }
    }
}

template <class T>
__global__ __launch_bounds__(256) void k_dst_rows(DstArgs<T> A) {
    dst_rows_body(A, blockIdx.x);
}

// first and last grid rows of a grid array: zero
template <class T>
__device__ void zero_edge_body(const ZeroArgs<T> &A, int blk) {
    if (A.done && *A.done) return;
    const int M = A.M;
    int i = blk * blockDim.x + threadIdx.x;
    if (i > M) return;
    const size_t last = (size_t)M * (M + 1) + i;
    A.grid[i] = zero<T>();
    A.grid[last] = zero<T>();
    if (A.upd) {
        A.upd[i] = lin2(A.upd_c0, zero<T>(), A.upd_c1, A.upd[i]);
        A.upd[last] = lin2(A.upd_c0, zero<T>(), A.upd_c1, A.upd[last]);
    }
}

// the Gamma part of the state update (ZeroArgs::upd_ag)
template <class T>
__device__ void gamma_update_body(const ZeroArgs<T> &A, int blk) {
    if (A.done && *A.done) return;
    const int i = blk * blockDim.x + threadIdx.x;
    if (i >= A.nb) return;
    A.upd_ag[i] = lin2(A.upd_c0, A.upd_g[i], A.upd_c1, A.upd_ag[i]);
}

// the b-solve's DST of f with, from the workgroups past the transform's nd,
// the corrections of f at the irregular nodes (independent work; one launch
// instead of two)
template <class T>
__global__ __launch_bounds__(256) void k_dst_rows_corr(DstArgs<T> A, CorrArgs<T> C, int nd) {
    if ((int)blockIdx.x < nd) dst_rows_body(A, blockIdx.x);
    else corrections_body(C, (int)blockIdx.x - nd);
}

// the DST of rows into a grid array with, from the workgroups past the
// transform's nd, the zeros of the grid's first and last rows (one launch
// instead of two; the two write disjoint rows)
template <class T>
__global__ __launch_bounds__(256) void k_dst_rows_grid(DstArgs<T> A, ZeroArgs<T> Z, int nd, int nz) {
    const int b = blockIdx.x;
    if (b < nd) dst_rows_body(A, b);
    else if (b < nd + nz) zero_edge_body(Z, b - nd);
    else gamma_update_body(Z, b - nd - nz);  // with a state update only
}

// ---------------------------------------------------------------------------
// Thomas coefficients.  With e_1 = 1/d, e_t = 1/(d - e_{t-1}) the forward
// sweep is x_t = e_t (x_{t-1} - rho_t) and the backward sweep
// U_t = e_t U_{t+1} + x_t.  e_t converges geometrically to the root of
// e = 1/(d - e) inside the unit disk; it is tabulated until it stops
// changing (relative 1e-17) and the limit is used afterwards.
// ---------------------------------------------------------------------------
// computed in FP64 (complex128) and stored in the solve precision S
template <class S>
__global__ void k_coef(int M, double kh2_re, double kh2_im, S *etab, S *elim, int32_t *tconv) {
    typedef typename High<S>::type H;
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = M - 1;
    if (k >= n) return;
    double s = sinpi((double)(k + 1) / (2.0 * M));
    H dk = from_re_im<H>(2.0 + 4.0 * s * s + kh2_re, kh2_im);
    H e = one<H>() / dk;
    int t = 0;
    for (; t < n; ++t) {
        etab[(size_t)t * n + k] = Conv<S>::from(e);
        H nx = one<H>() / (dk - e);
        H df = nx - e;
        if (abs2(df) <= 1e-34 * abs2(e)) { e = nx; ++t; break; }
        e = nx;
    }
    tconv[k] = t;
    elim[k] = Conv<S>::from(e);
}

// ---------------------------------------------------------------------------
// tridiagonal solves for MB consecutive modes per workgroup of MB*LANES
// threads; LANES lanes (one wavefront or half of one) share a mode, each
// owning C consecutive rows (LANES*C >= n).
//   phase A  the right-hand side rho_t = h^2 (rhat[t][k] + sum over the
//            irregular nodes q of row t of corr[q] sin(pi i_q k / M)) is
//            built in an LDS tile: the dense part (or zero) as MB-mode
//            contiguous row segments, then the sparse sums over segments of
//            at most kSegLen nodes of one row (all MB modes at once, so each
//            staged entry is read once), merged per row in a fixed order;
//   phase B  forward / backward recurrences as chunked affine scans with
//            wavefront shuffles, in place in the tile;
//   phase C  the tile is written out as contiguous MB-mode row segments.
// The tile index is t*MB + m + t/C: one element of padding per chunk keeps
// the lanes of phase B (stride C rows) off a single LDS bank.
// ---------------------------------------------------------------------------
// LDS per workgroup on gfx950: 160 KB
constexpr size_t kTriLdsMax = 163840;

// LDS slots (8 bytes each) of the tridiagonal kernels' sine table: the
// whole period sin(pi r / M), r = 0 .. 2M-1, in the tile kernel; the half
// period r = 0 .. M-1 in the register-row kernel, which reads it through
// sin_folded (the same values, one select more per read, half the LDS)
__host__ __device__ inline int tri_sine_slots(int M, bool folded) { return folded ? M : 2 * M; }

// Workgroups are dispatched to the 8 XCDs round-robin (workgroup b on XCD
// b mod 8).  xcd_tile maps workgroup b to a tile index so that each XCD
// owns one contiguous run of tiles (a bijection on [0, G) for any G): the
// mode groups written by one XCD are then adjacent, and the partial rows
// each workgroup writes merge into whole cache lines in that XCD's L2
// before they go to HBM.
__device__ inline int xcd_tile(int b, int G) {
    const int x = b & 7, i = b >> 3, per = G >> 3, rem = G & 7;
    const int first = x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per;
    return first + i;
}

template <int MB, int C>
__device__ inline int tidx(int t, int m) {
    return t * MB + m + t / C;
}

// T: the solve precision (double / cd, or float / cf for the mixed mode);
// the corrections arrive in FP64 (TC) and are rounded once when staged.
// STAGE: the sparse right-hand side and its segment tables are copied to
// LDS first; otherwise they are read from global memory.

constexpr int kCorrWin = 16;
// segment and row descriptors each thread of the tridiagonal kernel loads
// ahead (the rest, if any, are loaded where they are used)
constexpr int kPf = 2;
typedef int gi4 __attribute__((ext_vector_type(4)));

// Phase A of the sparse solves: the sums over every segment (at most kSegLen
// irregular nodes of one row) of corr[q] sin(pi i_q k / M) for the MB modes
// k = k0+1 .. k0+MB, into spart[segment * MB + mode].  Thread i of NT takes
// segments i, i + NT, ... (the first kPf from the descriptors it loaded
// ahead); four nodes per step keep several LDS round trips in flight, and
// each mode's terms are added in node order.  S is the sine table of
// tri_sine_slots: the whole period, or (FOLD) the half period read through
// sin_folded.
template <class T, class TC, int MB, int NT, bool STAGE, bool FOLD>
__device__ __forceinline__ void segment_sums(const gi4 (&sdesc)[kPf], const gmem<gi4> *__restrict__ seg_desc,
                                             int n_seg, int k0, int M, const typename Real<T>::type *S,
                                             const T *sval, const int32_t *scol, const gmem<TC> *__restrict__ corr,
                                             const gmem<int32_t> *__restrict__ irr_col, T *spart) {
#pragma clang fp contract(off)
    const int mask2M = 2 * M - 1;
    // one segment's sums, descriptor d = {first node, end node, row}
    auto seg_sum = [&](const gi4 d, int sg) {
        int q = d.x;
        const int q1 = d.y;
        T acc[MB];
#pragma unroll
        for (int mm = 0; mm < MB; ++mm) acc[mm] = zero<T>();
        for (; q + 4 <= q1; q += 4) {
            T cv[4];
            int col[4], idx[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                cv[u] = STAGE ? sval[q + u] : Conv<T>::from(gld(corr + (q + u)));
                col[u] = STAGE ? scol[q + u] : irr_col[q + u];
                idx[u] = (col[u] * (k0 + 1)) & mask2M;
            }
#pragma unroll
            for (int mm = 0; mm < MB; ++mm) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    acc[mm] = mad_(cv[u], FOLD ? sin_folded(S, idx[u], M) : S[idx[u]], acc[mm]);
                    idx[u] = (idx[u] + col[u]) & mask2M;
                }
            }
        }
        for (; q < q1; ++q) {
            const T cv = STAGE ? sval[q] : Conv<T>::from(gld(corr + (q)));
            const int col = STAGE ? scol[q] : irr_col[q];
            int idx = (col * (k0 + 1)) & mask2M;
#pragma unroll
            for (int mm = 0; mm < MB; ++mm) {
                acc[mm] = mad_(cv, FOLD ? sin_folded(S, idx, M) : S[idx], acc[mm]);
                idx = (idx + col) & mask2M;
            }
        }
#pragma unroll
        for (int mm = 0; mm < MB; ++mm) spart[sg * MB + mm] = acc[mm];
    };
#pragma unroll
    for (int r = 0; r < kPf; ++r) {
        const int sg = threadIdx.x + r * NT;
        if (sg < n_seg) seg_sum(sdesc[r], sg);
    }
    for (int sg = threadIdx.x + kPf * NT; sg < n_seg; sg += NT) seg_sum(seg_desc[sg], sg);
}

// Cross-lane moves for the scans of phase B, per element type: DPP moves
// within the wavefront (lanes whose source lies outside the pattern keep
// `old`) and reads of one lane's value by every lane.
__device__ __forceinline__ unsigned long long u64_of(double v) { return __builtin_bit_cast(unsigned long long, v); }
__device__ __forceinline__ double f64_of(unsigned long long u) { return __builtin_bit_cast(double, u); }

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double old, double v) {
    const unsigned long long o = u64_of(old), x = u64_of(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)o, (int)(unsigned)x, CTRL, 0xf, 0xf, false);
    const unsigned hi =
        (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)(o >> 32), (int)(unsigned)(x >> 32), CTRL, 0xf, 0xf, false);
    return f64_of(((unsigned long long)hi << 32) | lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float old, float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old), __builtin_bit_cast(int, v),
                                                                 CTRL, 0xf, 0xf, false));
}
__device__ __forceinline__ double lane_f64(double v, int l) {
    const unsigned long long x = u64_of(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)x, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(x >> 32), l);
    return f64_of(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ float lane_f32(float v, int l) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

template <class T> struct Xl;
template <> struct Xl<double> {
    template <int CTRL> __device__ static double dpp(double old, double v) { return dpp_f64<CTRL>(old, v); }
    __device__ static double at(double v, int l) { return lane_f64(v, l); }
};
template <> struct Xl<float> {
    template <int CTRL> __device__ static float dpp(float old, float v) { return dpp_f32<CTRL>(old, v); }
    __device__ static float at(float v, int l) { return lane_f32(v, l); }
};
template <> struct Xl<cd> {
    template <int CTRL> __device__ static cd dpp(cd old, cd v) {
        return make_cd(dpp_f64<CTRL>(old.x, v.x), dpp_f64<CTRL>(old.y, v.y));
    }
    __device__ static cd at(cd v, int l) { return make_cd(lane_f64(v.x, l), lane_f64(v.y, l)); }
};
template <> struct Xl<cf> {
    template <int CTRL> __device__ static cf dpp(cf old, cf v) {
        return make_cf(dpp_f32<CTRL>(old.x, v.x), dpp_f32<CTRL>(old.y, v.y));
    }
    __device__ static cf at(cf v, int l) { return make_cf(lane_f32(v.x, l), lane_f32(v.y, l)); }
};

// DPP controls (GFX9 encoding): row_shl:k 0x100+k, row_shr:k 0x110+k,
// wave_shl:1 0x130, wave_shr:1 0x138
constexpr int kDppRowShl = 0x100, kDppRowShr = 0x110, kDppWaveShl1 = 0x130, kDppWaveShr1 = 0x138;

// (A, B) <- (A, B) o (Ap, Bp) with (Ap, Bp) the map of lanes `CTRL` away
// (identity where there is none): y = A (Ap x + Bp) + B
template <class T, int CTRL>
__device__ __forceinline__ void compose_dpp(T &A, T &B) {
    const T Ap = Xl<T>::template dpp<CTRL>(one<T>(), A);
    const T Bp = Xl<T>::template dpp<CTRL>(zero<T>(), B);
    B = mad_(A, Bp, B);
    A = mul_(A, Ap);
}

// Phase B of the tridiagonal solves for one lane of a LANES-lane mode group
// (LANES = 64: the wavefront; 32: each half of it): v holds h^2 rho of the
// lane's C rows t0 .. t0+C-1 on entry and U^ on exit, e their Thomas
// coefficients (rows past n: v = e = 0).  The forward sweep
// x_t = e_t (x_{t-1} - rho_t) and the backward sweep U_t = e_t U_{t+1} + x_t
// are affine maps: each lane composes its rows' maps, the lanes' maps are
// composed in order (within rows of 16 lanes by DPP shifts, then across rows
// from the rows' totals read from their last / first lane), and each lane
// finishes its rows from the value carried in.
template <class T, int LANES, int C>
__device__ __forceinline__ void thomas_rows(T (&v)[C], const T (&e)[C], int lane, int t0, int n) {
#pragma clang fp contract(off)
    static_assert(LANES == 64 || LANES == 32, "mode groups of 32 or 64 lanes");
    const int row = (threadIdx.x & 63) >> 4;
    T A = one<T>(), B = zero<T>();
#pragma unroll
    for (int c = 0; c < C; ++c) {
        if (t0 + c < n) {
            B = mul_(e[c], B - v[c]);
            A = mul_(e[c], A);
        }
    }
    // forward: prefix over the lanes of each row of 16, then the rows before
    compose_dpp<T, kDppRowShr + 1>(A, B);
    compose_dpp<T, kDppRowShr + 2>(A, B);
    compose_dpp<T, kDppRowShr + 4>(A, B);
    compose_dpp<T, kDppRowShr + 8>(A, B);
    {
        const T A0 = Xl<T>::at(A, 15), B0 = Xl<T>::at(B, 15);
        const T A2 = Xl<T>::at(A, 47), B2 = Xl<T>::at(B, 47);
        T Ae = one<T>(), Be = zero<T>();
        if (LANES == 64) {
            const T A1 = Xl<T>::at(A, 31), B1 = Xl<T>::at(B, 31);
            const T B01 = mad_(A1, B0, B1), A01 = mul_(A1, A0);
            const T B012 = mad_(A2, B01, B2), A012 = mul_(A2, A01);
            if (row == 1) { Ae = A0; Be = B0; }
            if (row == 2) { Ae = A01; Be = B01; }
            if (row == 3) { Ae = A012; Be = B012; }
        } else {
            if (row == 1) { Ae = A0; Be = B0; }
            if (row == 3) { Ae = A2; Be = B2; }
        }
        B = mad_(A, Be, B);
    }
    T x = Xl<T>::template dpp<kDppWaveShr1>(zero<T>(), B);
    if (lane == 0) x = zero<T>();
#pragma unroll
    for (int c = 0; c < C; ++c) {
        x = mul_(e[c], x - v[c]);
        v[c] = x;
    }
    A = one<T>();
    B = zero<T>();
#pragma unroll
    for (int c = C - 1; c >= 0; --c) {
        B = mad_(e[c], B, v[c]);
        A = mul_(e[c], A);
    }
    // backward: suffix over the lanes of each row, then the rows after
    compose_dpp<T, kDppRowShl + 1>(A, B);
    compose_dpp<T, kDppRowShl + 2>(A, B);
    compose_dpp<T, kDppRowShl + 4>(A, B);
    compose_dpp<T, kDppRowShl + 8>(A, B);
    {
        const T A1 = Xl<T>::at(A, 16), B1 = Xl<T>::at(B, 16);
        const T A3 = Xl<T>::at(A, 48), B3 = Xl<T>::at(B, 48);
        T Ae = one<T>(), Be = zero<T>();
        if (LANES == 64) {
            const T A2 = Xl<T>::at(A, 32), B2 = Xl<T>::at(B, 32);
            const T B23 = mad_(A2, B3, B2), A23 = mul_(A2, A3);
            const T B123 = mad_(A1, B23, B1);
            if (row == 2) { Ae = A3; Be = B3; }
            if (row == 1) { Ae = A23; Be = B23; }
            if (row == 0) { Be = B123; Ae = mul_(A1, A23); }
        } else {
            if (row == 0) { Ae = A1; Be = B1; }
            if (row == 2) { Ae = A3; Be = B3; }
        }
        B = mad_(A, Be, B);
    }
    T y = Xl<T>::template dpp<kDppWaveShl1>(zero<T>(), B);
    if (lane == LANES - 1) y = zero<T>();
#pragma unroll
    for (int c = C - 1; c >= 0; --c) {
        y = mad_(e[c], y, v[c]);
        v[c] = y;
    }
}

template <class T, class TC, int MB, int LANES, int C, bool STAGE>
__device__ void tridiag_body(const TriArgs<T, TC> &A, int tile_idx) {
#pragma clang fp contract(off)
    typedef typename Real<T>::type R;
    const int M = A.M;
    const double h2 = A.h2;
    const gmem<T> *__restrict__ rhat = gview(A.rhat);
    const gmem<TC> *__restrict__ corr = gview(A.corr);
    const TriSparse &sp = A.sp;
    const gmem<int32_t> *__restrict__ irr_col = gview(sp.irr_col);
    const gmem<gi4> *__restrict__ seg_desc = (const gmem<gi4> *)gview(sp.seg_desc);
    const gmem<gi4> *__restrict__ row_desc = (const gmem<gi4> *)gview(sp.row_desc);
    const gmem<R> *__restrict__ sine = gview(A.sine);
    const gmem<T> *__restrict__ etab = gview(A.etab);
    const gmem<T> *__restrict__ elim = gview(A.elim);
    const gmem<int32_t> *__restrict__ tconv = gview(A.tconv);
    gmem<T> *__restrict__ uhat = gview(A.uhat);
    const gmem<int> *__restrict__ done = gview(A.done);
    extern __shared__ double lds[];
    constexpr int NT = MB * LANES;
    const int n = M - 1;
    if (done && *done) return;
    const int nnz = sp.nnz, n_act = sp.n_act, n_seg = sp.n_seg;
    R *S = reinterpret_cast<R *>(lds);                   // the sine table, a whole period
    T *tile = reinterpret_cast<T *>(lds + tri_sine_slots(M, false));  // n*MB + n/C + 1
    const int tile_len = n * MB + n / C + 1;
    T *spart = tile + tile_len;                          // n_seg*MB partial sums
    // staged sparse right-hand side: values and columns
    const bool sparse = corr != nullptr;
    T *sval = spart + (sparse ? n_seg * MB : 0);
    int32_t *scol = reinterpret_cast<int32_t *>(sval + (STAGE ? nnz : 0));
    const int k0 = tile_idx * MB;
    // the descriptors of the thread's first kPf segments and rows, loaded
    // before anything else so that the sums and the merge below start
    // without a dependent round trip to memory
    gi4 sdesc[kPf], rdesc[kPf];
    if (sparse) {
#pragma unroll
        for (int r = 0; r < kPf; ++r) {
            const int g = threadIdx.x + r * NT, a = threadIdx.x + r * NT;
            sdesc[r] = seg_desc[g < n_seg ? g : 0];
            rdesc[r] = row_desc[a < n_act ? a : 0];
        }
    }
    const int lane = threadIdx.x % LANES;
    const int m = threadIdx.x / LANES;
    const int k = k0 + m;
    const int t0 = lane * C;
    int tc = 0;
    T lim = zero<T>();
    if (k < n) {
        tc = tconv[k];
        lim = gld(elim + k);
    }
    // sine table and staging: loads batched so that several are in flight
    const int nsq = tri_sine_slots(M, false);
    for (int q0 = threadIdx.x; q0 < nsq; q0 += 4 * NT) {
        R v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (q0 + u * NT < nsq) v[u] = sine[q0 + u * NT];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (q0 + u * NT < nsq) S[q0 + u * NT] = v[u];
    }
    if (STAGE && corr) {
        for (int q0 = threadIdx.x; q0 < nnz; q0 += 4 * NT) {
            TC v[4];
            int32_t c[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int q = q0 + u * NT;
                if (q < nnz) {
                    v[u] = gld(corr + (q));
                    c[u] = irr_col[q];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int q = q0 + u * NT;
                if (q < nnz) {
                    sval[q] = Conv<T>::from(v[u]);
                    scol[q] = c[u];
                }
            }
        }
    }
    // dense part (or zero) of the right-hand side
    for (int p = threadIdx.x; p < n * MB; p += NT) {
        const int t = p / MB, mm = p - t * MB;
        tile[tidx<MB, C>(t, mm)] = (rhat && k0 + mm < n) ? gld(rhat + (size_t)t * n + k0 + mm) : zero<T>();
    }
    __syncthreads();
    // Thomas coefficients of phase B: loads in flight during phase A
    T e[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int t = t0 + c;
        e[c] = (t < tc && t < n) ? gld(etab + (size_t)t * n + k) : lim;
    }
    // phase A: sparse sums.  Each thread sums one segment (at most kSegLen
    // irregular nodes of one row) for all MB modes; four nodes per step keep
    // several LDS round trips in flight.  Then one thread per row adds its
    // segments' partial sums in order, so the result does not depend on
    // the schedule.
    if (sparse) {
        segment_sums<T, TC, MB, NT, STAGE, false>(sdesc, seg_desc, n_seg, k0, M, S, sval, scol, corr, irr_col, spart);
        __syncthreads();
        // one row's segments added in order, descriptor d = {row, first
        // segment, end segment}
        auto row_merge = [&](const gi4 d) {
            const int t = d.x, s0 = d.y, s1 = d.z;
            T acc[MB];
#pragma unroll
            for (int mm = 0; mm < MB; ++mm) acc[mm] = spart[s0 * MB + mm];
            for (int sg = s0 + 1; sg < s1; ++sg)
#pragma unroll
                for (int mm = 0; mm < MB; ++mm) acc[mm] += spart[sg * MB + mm];
#pragma unroll
            for (int mm = 0; mm < MB; ++mm) tile[tidx<MB, C>(t, mm)] += acc[mm];
        };
#pragma unroll
        for (int r = 0; r < kPf; ++r) {
            const int a = threadIdx.x + r * NT;
            if (a < n_act) row_merge(rdesc[r]);
        }
        for (int a = threadIdx.x + kPf * NT; a < n_act; a += NT) row_merge(row_desc[a]);
    }
    __syncthreads();
    // phase B
    if (k < n) {
        // the lane's rows in registers for all four passes (rows past n: 0 with
        // e = 0, which leaves every composite unchanged)
        T v[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const bool ok = t0 + c < n;
            v[c] = ok ? tile[tidx<MB, C>(t0 + c, m)] * (R)h2 : zero<T>();
            if (!ok) e[c] = zero<T>();
        }
        thomas_rows<T, LANES, C>(v, e, lane, t0, n);
#pragma unroll
        for (int c = C - 1; c >= 0; --c)
            if (t0 + c < n) tile[tidx<MB, C>(t0 + c, m)] = v[c];
    }
    __syncthreads();
    // phase C
    for (int p = threadIdx.x; p < n * MB; p += NT) {
        const int t = p / MB, mm = p - t * MB;
        if (k0 + mm < n) gst(uhat + (size_t)t * n + k0 + mm, tile[tidx<MB, C>(t, mm)]);
    }
}

template <class T, class TC, int MB, int LANES, int C, bool STAGE>
__global__ __launch_bounds__(MB *LANES) void k_tridiag(TriArgs<T, TC> A) {
    tridiag_body<T, TC, MB, LANES, C, STAGE>(A, xcd_tile(blockIdx.x, gridDim.x));
}

// ---------------------------------------------------------------------------
// The same solves for a sparse right-hand side without the LDS tile: after
// phase A's segment sums each lane adds the partial sums of its own C rows
// (row t's segments row_span[t], in the order of the row merge above)
// straight into registers, runs the same scans, and the results leave
// through a small LDS buffer, CH rows per lane at a time, as the same MB-mode
// row segments.  Every value is formed by the same operations in the same
// order as in tridiag_body; the LDS shrinks from the n*MB tile to the larger
// of the partial sums and the buffer, so more workgroups share a CU.
// 64-lane mode groups only.
// ---------------------------------------------------------------------------
template <int C>
struct RowsOut {
    static constexpr int CH = C < 4 ? C : 4;  // rows per lane per output chunk
};

template <class T, int MB, int C>
constexpr size_t rows_obuf_bytes() {
    return (size_t)RowsOut<C>::CH * 64 * (MB > 1 ? MB + 1 : 1) * sizeof(T);
}

typedef int gi2 __attribute__((ext_vector_type(2)));

// DENSE: the right-hand side also has the dense part rhat (b-solve, final
// solve), each lane reading its own rows of it (batched launches only)
template <class T, class TC, int MB, int C, bool STAGE, bool DENSE>
__device__ void tridiag_rows_body(const TriArgs<T, TC> &A, int tile_idx) {
#pragma clang fp contract(off)
    typedef typename Real<T>::type R;
    constexpr int LANES = 64, NT = MB * LANES;
    constexpr int CH = RowsOut<C>::CH;
    constexpr int OST = MB > 1 ? MB + 1 : 1;  // padded slot stride of the buffer
    const int M = A.M;
    const double h2 = A.h2;
    const gmem<TC> *__restrict__ corr = gview(A.corr);
    const TriSparse &sp = A.sp;
    const gmem<int32_t> *__restrict__ irr_col = gview(sp.irr_col);
    const gmem<gi4> *__restrict__ seg_desc = (const gmem<gi4> *)gview(sp.seg_desc);
    const gmem<gi2> *__restrict__ row_span = (const gmem<gi2> *)gview(sp.row_span);
    const gmem<R> *__restrict__ sine = gview(A.sine);
    const gmem<T> *__restrict__ etab = gview(A.etab);
    const gmem<T> *__restrict__ elim = gview(A.elim);
    const gmem<int32_t> *__restrict__ tconv = gview(A.tconv);
    gmem<T> *__restrict__ uhat = gview(A.uhat);
    const gmem<int> *__restrict__ done = gview(A.done);
    extern __shared__ double lds[];
    const int n = M - 1;
    if (done && *done) return;
    const int nnz = sp.nnz, n_seg = sp.n_seg;
    R *S = reinterpret_cast<R *>(lds);                   // the sine table, half a period
    T *spart = reinterpret_cast<T *>(lds + tri_sine_slots(M, true));  // n_seg*MB partial sums
    T *obuf = spart;                                     // later: the output chunks
    T *sval = spart + n_seg * MB;
    int32_t *scol = reinterpret_cast<int32_t *>(sval + (STAGE ? nnz : 0));
    const int k0 = tile_idx * MB;
    const int lane = threadIdx.x % LANES;
    const int m = threadIdx.x / LANES;
    const int k = k0 + m;
    const int t0 = lane * C;
    gi4 sdesc[kPf];
#pragma unroll
    for (int r = 0; r < kPf; ++r) {
        const int g = threadIdx.x + r * NT;
        sdesc[r] = seg_desc[g < n_seg ? g : 0];
    }
    // segment spans of the lane's rows (the table holds 64*C rows)
    gi2 rsp[C];
#pragma unroll
    for (int c = 0; c < C; ++c) rsp[c] = row_span[t0 + c];
    // the dense part of the lane's rows: every load issued at a clamped,
    // in-bounds index and masked afterwards
    T rh[DENSE ? C : 1];
    if constexpr (DENSE) {
        const gmem<T> *__restrict__ rhat = gview(A.rhat);
        const int kc = k < n ? k : n - 1;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int t = t0 + c;
            const T x = gld(rhat + (size_t)(t < n ? t : n - 1) * n + kc);
            rh[c] = (t < n && k < n) ? x : zero<T>();
        }
    }
    int tc = 0;
    T lim = zero<T>();
    if (k < n) {
        tc = tconv[k];
        lim = gld(elim + k);
    }
    const int nsq = tri_sine_slots(M, true);
    for (int q0 = threadIdx.x; q0 < nsq; q0 += 4 * NT) {
        R v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (q0 + u * NT < nsq) v[u] = sine[q0 + u * NT];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (q0 + u * NT < nsq) S[q0 + u * NT] = v[u];
    }
    if (STAGE) {
        for (int q0 = threadIdx.x; q0 < nnz; q0 += 4 * NT) {
            TC v[4];
            int32_t c[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int q = q0 + u * NT;
                if (q < nnz) {
                    v[u] = gld(corr + (q));
                    c[u] = irr_col[q];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int q = q0 + u * NT;
                if (q < nnz) {
                    sval[q] = Conv<T>::from(v[u]);
                    scol[q] = c[u];
                }
            }
        }
    }
    __syncthreads();
    T e[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int t = t0 + c;
        e[c] = (t < tc && t < n) ? gld(etab + (size_t)t * n + k) : lim;
    }
    // phase A
    segment_sums<T, TC, MB, NT, STAGE, true>(sdesc, seg_desc, n_seg, k0, M, S, sval, scol, corr, irr_col, spart);
    __syncthreads();
    // phase B: the lane's rows from the partial sums (0, or the dense part,
    // plus the row's segments in order, as the tile kernel's tile plus its
    // row merge), then the scans
    // every row's first partial sum read at once (clamped: a row without
    // nodes reads a valid entry and ignores it), later segments after
    T v[C], first[C];
#pragma unroll
    for (int c = 0; c < C; ++c) first[c] = spart[min(rsp[c].x, n_seg - 1) * MB + m];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        T acc = zero<T>();
        if constexpr (DENSE) acc = rh[c];
        const int s0 = rsp[c].x, s1 = rsp[c].y;
        if (s0 < s1) {
            T a = first[c];
            for (int sg = s0 + 1; sg < s1; ++sg) a += spart[sg * MB + m];
            acc += a;
        }
        const bool ok = t0 + c < n;
        v[c] = ok ? acc * (R)h2 : zero<T>();
        if (!ok) e[c] = zero<T>();
    }
    if (k < n) thomas_rows<T, LANES, C>(v, e, lane, t0, n);
    // phase C: CH rows per lane at a time through the buffer (which
    // overlays the partial sums: the first barrier also ends their reads)
#pragma unroll
    for (int cb = 0; cb < C; cb += CH) {
        __syncthreads();
#pragma unroll
        for (int cc = 0; cc < CH; ++cc) obuf[(cc * LANES + lane) * OST + m] = v[cb + cc];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < CH; ++r) {
            const int p = threadIdx.x + r * NT;  // < CH * LANES * MB
            const int slot = p / MB, mm = p - slot * MB;
            const int t = (slot % LANES) * C + cb + slot / LANES;
            if (t < n && k0 + mm < n) gst(uhat + (size_t)t * n + k0 + mm, obuf[slot * OST + mm]);
        }
    }
}

template <class T, class TC, int MB, int C, bool STAGE>
__global__ __launch_bounds__(MB * 64) void k_tridiag_rows(TriArgs<T, TC> A) {
    tridiag_rows_body<T, TC, MB, C, STAGE, false>(A, xcd_tile(blockIdx.x, gridDim.x));
}

// ---------------------------------------------------------------------------
// U at listed nodes: one wavefront per node, U = (2/M) sum_k U^[t][k]
// sin(pi i k / M).  nodes: linear grid indices (interior nodes only).
// ---------------------------------------------------------------------------
// T: precision of U^ and of the sum; the result is stored in FP64 (TO)
// Sum over modes of one row against the sine of one column i:
// sum_k row[k] sin(pi i (k+1) / M), lanes taking k = lane + 64 j in turn
// (the order of every stencil evaluation, so all of them agree bit for
// bit).  The table S holds sin(pi q / M), q < 2M (M a power of two).  The
// sine of the lane's angle a_j = a + b_j, a = (lane+1) i and b_j = 64 j i,
// is sin a cos b_j + cos a sin b_j: two lane-dependent table reads per
// column and two uniform ones per step instead of a scattered read per
// mode (cos x read as sin(x + pi/2)).  get(j) returns row[lane + 64 j];
// KR > 0 unrolls KR steps (values held in registers), KR = 0 loops.
template <int KR, class T, class SP, class R, class G>
__device__ __forceinline__ T mode_sum(SP S, const cmem<R> *scu, int M, int n, int i, int lane, const G &get) {
    const int mask2M = 2 * M - 1, quarter = M >> 1;
    const int ia = (i * (lane + 1)) & mask2M;
    R sa, ca;
    if constexpr (KR > 0) {
        // M = 64 KR, and S extends a quarter period past 2M
        sa = S[ia];
        ca = S[ia + 32 * KR];
    } else {
        sa = S[ia];
        ca = S[(ia + quarter) & mask2M];
    }
    // the step angle 64 i j (mod 2M) is 64 m with m = i j mod max(1, M/32):
    // its sine and cosine come from the step table, the same for every lane
    // of the wavefront (i is uniform), so they load into scalar registers
    const int mu = (KR > 0 ? 2 * KR : max(1, M >> 5)) - 1;
    T acc = zero<T>();
    if constexpr (KR > 0) {
        // get(j) is zero past the last mode, so every step adds exactly what
        // the guarded loop adds
#pragma unroll
        for (int j = 0; j < KR; ++j) {
            const int m = (i * j) & mu;
            const R sv = fma(ca, (R)scu[2 * m], sa * (R)scu[2 * m + 1]);
            acc += get(j) * sv;
        }
    } else {
        for (int j = 0; 64 * j < n; ++j) {
            const int m = (i * j) & mu;
            const R sv = fma(ca, (R)scu[2 * m], sa * (R)scu[2 * m + 1]);
            if (lane + 64 * j < n) acc += get(j) * sv;
        }
    }
    return acc;
}

template <class T, class TO>
__device__ void eval_nodes_body(const EvalArgs<T, TO> &A, int blk) {
    typedef typename Real<T>::type R;
    const int M = A.M, nnodes = A.nnodes, node_stride = A.node_stride;
    const int32_t *__restrict__ nodes = A.nodes;
    const T *__restrict__ uhat = A.uhat;
    const R *__restrict__ sine = A.sine;
    TO *__restrict__ out = A.out;
    if (A.done && *A.done) return;
    const int lane = threadIdx.x & 63;
    const int p = blk * 4 + (threadIdx.x >> 6);
    if (p >= nnodes) return;
    const int n = M - 1;
    // nodes of a stencil record are 6 consecutive int32 followed by the rest of
    // the record; node_stride is the record size in int32 units
    // one node per wavefront: uniform, kept in scalar registers
    int node = __builtin_amdgcn_readfirstlane(nodes[(size_t)(p / 6) * node_stride + (p % 6)]);
    int i = node % (M + 1), j = node / (M + 1);
    const T *row = uhat + (size_t)(j - 1) * n;
    T acc = mode_sum<0, T>(gview(sine), cview(A.scu), M, n, i, lane, [&](int q) { return gld(gview(row) + lane + 64 * q); });
    acc = wave_sum(acc);
    if (lane == 0) out[p] = to_high(acc * (R)(2.0 / M));
}

template <class T, class TO>
__global__ __launch_bounds__(256) void k_eval_nodes(EvalArgs<T, TO> A) {
    // each XCD takes one run of consecutive nodes, which lie on one arc of
    // the boundary: the rows of U^ that arc needs are then fetched into one
    // XCD's L2, not into all eight
    eval_nodes_body(A, xcd_tile(blockIdx.x, gridDim.x));
}

// corrections of a density with the merged operator, one thread per node
template <class TC>
__device__ void corr_phi_body(const CorrPhiArgs<TC> &A, int blk) {
    const TC *__restrict__ phi = A.phi;
    const int Nb = A.Nb, nnz = A.nnz;
    const TC *__restrict__ mcoef = A.mcoef;
    const int32_t *__restrict__ mbase = A.mbase;
    TC *__restrict__ corr = A.corr;
    if (A.done && *A.done) return;
    const int q = blk * blockDim.x + threadIdx.x;
    if (q >= nnz) return;
    const int b = mbase[q];
    TC acc = A.base ? A.base[q] : zero<TC>();
#pragma unroll
    for (int o = 0; o < kCorrWin; ++o) {
        int idx = b + o;
        if (idx >= Nb) idx -= Nb;
        acc += mcoef[(size_t)o * nnz + q] * phi[idx];
    }
    corr[q] = acc;
}

// With copy_out, the workgroups past those of the corrections copy the
// density there (one launch instead of two)
template <class TC>
__global__ __launch_bounds__(64) void k_corr_phi(CorrPhiArgs<TC> A) {
    const int nbc = (A.nnz + 63) / 64;
    if ((int)blockIdx.x < nbc) {
        corr_phi_body(A, blockIdx.x);
        return;
    }
    if (A.done && *A.done) return;
    const int k = ((int)blockIdx.x - nbc) * 64 + (int)threadIdx.x;
    if (k < A.Nb) A.copy_out[k] = A.phi[k];
}

// K phi at the collocation points, one workgroup of six wavefronts per
// point: wavefront p evaluates the grid solution at stencil node p (as
// k_eval_nodes: U = (2/M) sum_k U^[t][k] sin(pi i k / M), summed in the
// precision of U^ and stored in FP64), then one thread forms the extraction
// U+(z_k) = sum_p w6[k][p] U_p + sum_o bop[k][o] phi[k-2+o] in FP64 (the
// compact form of the six-point rule with the jump terms of the outside
// nodes, eq. 3.36).
// KR > 0: M = 64 KR, the row's modes loaded into registers at once (the
// same sums as KR = 0, which loops over the modes)
template <class T, class TO, int KR>
__device__ void eval_extract_body(const EvxArgs<T, TO> &A, int blk) {
    typedef typename Real<T>::type R;
    const int M = A.M, Nb = A.Nb, node_stride = A.node_stride;
    const int32_t *__restrict__ nodes = A.nodes;
    const T *__restrict__ uhat = A.uhat;
    const R *__restrict__ sine = A.sine;
    const double *__restrict__ w6 = A.w6;
    const TO *__restrict__ bop = A.bop;
    const TO *__restrict__ phi = A.phi;
    TO *__restrict__ kv = A.kv;
    __shared__ TO su[6];
    if (A.done && *A.done) return;
    const int lane = threadIdx.x & 63, p = threadIdx.x >> 6;
    const int k = blk;
    const int n = M - 1;
    // the extraction's weights and density window, loaded by thread 0 now so
    // that they arrive during the row sums
    double wq[6];
    TO bq[5], fq[5];
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < 6; ++q) wq[q] = w6[6 * k + q];
#pragma unroll
        for (int o = 0; o < 5; ++o) {
            int idx = k - 2 + o;
            idx = idx < 0 ? idx + Nb : (idx >= Nb ? idx - Nb : idx);
            bq[o] = bop[5 * k + o];
            fq[o] = phi[idx];
        }
    }
    const int node = __builtin_amdgcn_readfirstlane(nodes[(size_t)k * node_stride + p]);
    const int i = node % (M + 1);
    const T *row = uhat + (size_t)(node / (M + 1) - 1) * n;
    T acc;
    if constexpr (KR > 0) {
        T v[KR];
#pragma unroll
        for (int j = 0; j < KR; ++j) {
            const int q = lane + 64 * j;
            const T x = gld(gview(row) + min(q, n - 1));
            v[j] = q < n ? x : zero<T>();
        }
        acc = mode_sum<KR, T>(gview(sine), cview(A.scu), M, n, i, lane, [&](int jj) { return v[jj]; });
    } else {
        acc = mode_sum<0, T>(gview(sine), cview(A.scu), M, n, i, lane,
                             [&](int q) { return gld(gview(row) + lane + 64 * q); });
    }
    acc = wave_sum(acc);
    if (lane == 0) su[p] = to_high(acc * (R)(2.0 / M));
    __syncthreads();
    if (threadIdx.x == 0) {
        TO r = zero<TO>();
#pragma unroll
        for (int q = 0; q < 6; ++q) r = mad_(su[q], wq[q], r);
#pragma unroll
        for (int o = 0; o < 5; ++o) r = mad_(bq[o], fq[o], r);
        kv[k] = r;
    }
}

template <class T, class TO, int KR>
__global__ __launch_bounds__(384) void k_eval_extract(EvxArgs<T, TO> A) {
    // one run of consecutive collocation points (one arc) per XCD, as in
    // k_eval_nodes
    eval_extract_body<T, TO, KR>(A, xcd_tile(blockIdx.x, gridDim.x));
}

// the register-row form of the evaluation for M = 64 .. 1024, the loop above
template <class F>
void evx_dispatch(int M, const F &f) {
    switch (M) {
        case 64: f.template go<1>(); break;
        case 128: f.template go<2>(); break;
        case 256: f.template go<4>(); break;
        case 512: f.template go<8>(); break;
        case 1024: f.template go<16>(); break;
        default: f.template go<0>(); break;
    }
}

template <class T, class TO>
struct EvxLaunch {
    EvxArgs<T, TO> A;
    int blocks;
    hipStream_t s;
    template <int KR>
    void go() const {
        k_eval_extract<T, TO, KR><<<blocks, 384, 0, s>>>(A);
    }
};

// The b-solve's stencil values and general extraction in one launch: one
// workgroup of six wavefronts per collocation point; wavefront p evaluates
// stencil node p (the sums of k_eval_nodes, as in k_eval_extract), thread 0
// forms U+ with the jumps of f and the boundary data (as k_extract) from the
// six values in LDS.
template <class T, int KR>
__device__ void eval_extract_gen_body(const EvalArgs<T, T> &E, const ExtArgs<T> &X, int blk) {
    typedef typename Real<T>::type R;
    __shared__ T su[6];
    const int M = E.M, n = M - 1;
    const int lane = threadIdx.x & 63, p = threadIdx.x >> 6;
    const int k = blk;
    const int node = __builtin_amdgcn_readfirstlane(E.nodes[(size_t)k * E.node_stride + p]);
    const int i = node % (M + 1);
    const T *row = E.uhat + (size_t)(node / (M + 1) - 1) * n;
    T acc;
    if constexpr (KR > 0) {
        T v[KR];
#pragma unroll
        for (int j = 0; j < KR; ++j) {
            const int q = lane + 64 * j;
            const T x = gld(gview(row) + min(q, n - 1));
            v[j] = q < n ? x : zero<T>();
        }
        acc = mode_sum<KR, T>(gview(E.sine), cview(E.scu), M, n, i, lane, [&](int jj) { return v[jj]; });
    } else {
        acc = mode_sum<0, T>(gview(E.sine), cview(E.scu), M, n, i, lane,
                             [&](int q) { return gld(gview(row) + lane + 64 * q); });
    }
    acc = wave_sum(acc);
    if (lane == 0) su[p] = acc * (R)(2.0 / M);
    __syncthreads();
    if (threadIdx.x == 0) extract_point(X, k, [&](int q) { return su[q]; });
}

template <class T, int KR>
__global__ __launch_bounds__(384) void k_eval_extract_gen(EvalArgs<T, T> E, ExtArgs<T> X) {
    eval_extract_gen_body<T, KR>(E, X, xcd_tile(blockIdx.x, gridDim.x));
}

template <class T>
struct EvxGenLaunch {
    EvalArgs<T, T> E;
    ExtArgs<T> X;
    int blocks;
    hipStream_t s;
    template <int KR>
    void go() const {
        k_eval_extract_gen<T, KR><<<blocks, 384, 0, s>>>(E, X);
    }
};


// Grid values at the stencil nodes by rows: U = (2/M) sum_k U^[t][k]
// sin(pi i k / M) at each distinct stencil node (t, i), in the same sum and
// reduction order as k_eval_nodes.  Each wavefront takes kErowRows/4 rows
// in turn: it holds the row's n modes in registers (mode k = lane + 64 j in
// slot j, KR >= n/64 slots), forms the sum for each node of the row, and
// writes it to every stencil entry of that node.  Each needed row is read
// once and the sine table is staged once per workgroup.
template <class T, class TO, int KR>
__device__ void eval_rows_body(const ErowArgs<T, TO> &A, int blk) {
    typedef typename Real<T>::type R;
    constexpr int RW = kErowRows / 4;  // rows per wavefront
    if (A.done && *gview(A.done)) return;
    extern __shared__ double lds[];
    constexpr int M = 64 * KR, n = M - 1;  // the launch is per class of equal M
    const int n_rows = A.n_rows;
    const gmem<int32_t> *__restrict__ erow_t = gview(A.erow_t);
    const gmem<int32_t> *__restrict__ erow_ptr = gview(A.erow_ptr);
    const gmem<int32_t> *__restrict__ erow_col = gview(A.erow_col);
    const gmem<T> *__restrict__ uhat = gview(A.uhat);
    const gmem<R> *__restrict__ sine = gview(A.sine);
    const cmem<R> *__restrict__ scu = cview(A.scu);
    gmem<TO> *__restrict__ ust = gview(A.ust);
    R *S = reinterpret_cast<R *>(lds);
    int32_t *scol = reinterpret_cast<int32_t *>(S + 2 * M + M / 2);  // kErowCols node columns
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r0 = blk * kErowRows + w;  // the wavefront's rows: r0 + 4 q, q < RW
    // Every global load below is issued unconditionally at a clamped,
    // in-bounds index and masked afterwards, and the sums read only LDS:
    // loads under a branch, or loads between the row prefetch and its use,
    // make the compiler wait for all outstanding loads (the counter is in
    // order), which would serialise the prefetch.  Row indices and node
    // ranges of the wavefront's rows, one per lane (n_rows >= 1):
    const int rl = min(r0 + 4 * min(lane, RW - 1), n_rows - 1);
    const int t_l = erow_t[rl], p0_l = erow_ptr[rl], p1_l = erow_ptr[rl + 1];
    // the workgroup's nodes are the contiguous range [P0, P1)
    const int P0 = erow_ptr[min(blk * kErowRows, n_rows - 1)];
    const int P1 = erow_ptr[min((blk + 1) * kErowRows, n_rows)];
    auto load_row = [&](int q, T (&dst)[KR]) {
        const gmem<T> *src = uhat + (size_t)__shfl(t_l, q) * n;
#pragma unroll
        for (int j = 0; j < KR; ++j) {
            const int k = lane + 64 * j;
            const T x = gld(src + min(k, n - 1));
            dst[j] = k < n ? x : zero<T>();
        }
    };
    T v[KR], vn[KR];
    load_row(0, v);
    // sine table and node columns, loads batched so that several are in flight
    // (the table repeats its first quarter period after 2M)
    constexpr int SL = 2 * M + M / 2;
    for (int q0 = threadIdx.x; q0 < SL; q0 += 4 * 256) {
        R s4[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) s4[u] = sine[min(q0 + u * 256, SL - 1) & (2 * M - 1)];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (q0 + u * 256 < SL) S[q0 + u * 256] = s4[u];
    }
    for (int q = threadIdx.x; q < P1 - P0; q += 256) scol[q] = erow_col[P0 + q];
    __syncthreads();
    const R scale = (R)(2.0 / M);
#pragma unroll
    for (int q = 0; q < RW; ++q) {
        if (r0 + 4 * q >= n_rows) break;
        // next row's modes load during this row's sums (the last row reloads
        // a clamped row, unused)
        const bool more = q + 1 < RW && r0 + 4 * (q + 1) < n_rows;
        if (q + 1 < RW) load_row(q + 1, vn);
        const int p0 = __shfl(p0_l, q), p1 = __shfl(p1_l, q);
        for (int c = p0; c < p1; ++c) {
            // uniform over the wavefront: scalar index arithmetic
            const int i = __builtin_amdgcn_readfirstlane(scol[c - P0]);
            T acc = mode_sum<KR, T>(S, scu, M, n, i, lane, [&](int jj) { return v[jj]; });
            acc = wave_sum(acc);
            // every lane holds the sum: all write the same value
            gst(ust + c, to_high(acc * scale));
        }
        if (more) {
#pragma unroll
            for (int j = 0; j < KR; ++j) v[j] = vn[j];
        }
    }
}

// K phi at collocation point k from its six stencil values: the extraction
// sum_p w6[k][p] U_p + sum_o bop[k][o] phi[k-2+o] (as in k_eval_extract)
template <class T>
__device__ void extract_merged_body(const ExmArgs<T> &A, int blk) {
    if (A.done && *gview(A.done)) return;
    const int k = blk * blockDim.x + threadIdx.x, Nb = A.Nb;
    if (k >= Nb) return;
    const gmem<T> *__restrict__ ust = gview(A.ust);
    const gmem<int32_t> *__restrict__ nid = gview(A.nid);
    const gmem<double> *__restrict__ w6 = gview(A.w6);
    const gmem<T> *__restrict__ bop = gview(A.bop);
    const gmem<T> *__restrict__ phi = gview(A.phi);
    T r = zero<T>();
#pragma unroll
    for (int q = 0; q < 6; ++q) r = mad_(gld(ust + nid[6 * k + q]), (double)w6[6 * k + q], r);
#pragma unroll
    for (int o = 0; o < 5; ++o) {
        int idx = k - 2 + o;
        idx = idx < 0 ? idx + Nb : (idx >= Nb ? idx - Nb : idx);
        r = mad_(gld(bop + 5 * k + o), gld(phi + idx), r);
    }
    gst(gview(A.kv) + k, r);
}

template <class T>
__global__ __launch_bounds__(256) void k_extract_merged(ExmArgs<T> A) {
    extract_merged_body(A, blockIdx.x);
}

// argument blocks and launch shapes shared by the single and batched paths
template <class T> T coef_of(double re, double im);
template <> double coef_of<double>(double re, double) { return re; }
template <> cd coef_of<cd>(double re, double im) { return make_cd(re, im); }

template <class T>
DstArgs<T> dst_args(kfbi_domain *d, const void *in, bool in_grid, const uint8_t *mask, void *out, bool out_grid,
                    double scale, const int *done) {
    DstArgs<T> A;
    A.M = d->M;
    A.logN2 = 0;
    while ((1 << A.logN2) < 2 * d->M) ++A.logN2;
    A.in = (const T *)in;
    A.in_grid = in_grid ? 1 : 0;
    A.mask = mask;
    A.out = (T *)out;
    A.out_grid = out_grid ? 1 : 0;
    A.scale = scale;
    A.twiddle = d->twiddle;
    A.done = done;
    A.upd = nullptr;
    A.upd_c0 = zero<T>();
    A.upd_c1 = zero<T>();
    return A;
}
template <class T>
int dst_blocks(int M) {
    return sizeof(T) == sizeof(cd) ? M - 1 : M / 2;
}
inline size_t dst_lds(int M) { return (size_t)2 * M * sizeof(double2); }

template <class T>
int launch_dst(kfbi_domain *d, const void *in, bool in_grid, const uint8_t *mask, void *out,
               bool out_grid, double scale, const int *done = nullptr, const GridUpdate *up = nullptr) {
    const int M = d->M, n = M - 1;
    DstArgs<T> A = dst_args<T>(d, in, in_grid, mask, out, out_grid, scale, done);
    const int ps = prof_begin(d);
    const int nd = dst_blocks<T>(M), nz = (M + 1 + 255) / 256;
    if (out_grid) {
        ZeroArgs<T> Z{M, (T *)out, done};
        int ng = 0;  // workgroups of the Gamma part of a state update
        if (up) {
            A.upd = Z.upd = (T *)up->a;
            A.upd_c0 = Z.upd_c0 = coef_of<T>(up->c0r, up->c0i);
            A.upd_c1 = Z.upd_c1 = coef_of<T>(up->c1r, up->c1i);
            Z.upd_g = (const T *)up->g;
            Z.upd_ag = (T *)up->ag;
            Z.nb = d->Nb;
            ng = (d->Nb + 255) / 256;
        }
        k_dst_rows_grid<T><<<nd + nz + ng, 256, dst_lds(M), d->stream>>>(A, Z, nd, nz);
    } else
        k_dst_rows<T><<<nd, 256, dst_lds(M), d->stream>>>(A);
    KFBI_CHECK_LAUNCH();
    {
        const double es = sizeof(T), nn = (double)n * n, grid = (double)(M + 1) * (M + 1);
        const double bytes = in_grid ? es * (nn + nn) + (mask ? nn : 0.0) : es * (nn + grid);
        prof_end(d, ps, in_grid ? KFBI_K_DST : KFBI_K_IDST, bytes);
    }
    return KFBI_OK;
}

template <class TC>
CorrPhiArgs<TC> corr_phi_args(kfbi_domain *d, const void *phi, void *corr, const int *done,
                              const void *base = nullptr, void *copy_out = nullptr) {
    return CorrPhiArgs<TC>{(const TC *)phi, d->Nb,  d->n_irr, (const TC *)d->mcoef, d->mbase, (TC *)corr, done,
                           (const TC *)base, (TC *)copy_out};
}

template <class T, class TO>
EvxArgs<T, TO> evx_args(kfbi_domain *d, const void *uhat, const void *phi, void *kv, const int *done) {
    typedef typename Real<T>::type R;
    const bool low = sizeof(T) < sizeof(TO);
    EvxArgs<T, TO> A;
    A.M = d->M;
    A.Nb = d->Nb;
    A.node_stride = (int)(sizeof(Stencil) / sizeof(int32_t));
    A.nodes = reinterpret_cast<const int32_t *>(d->st);
    A.uhat = (const T *)uhat;
    A.sine = low ? (const R *)d->sine32 : (const R *)d->sine;
    A.scu = low ? (const R *)d->scu32 : (const R *)d->scu;
    A.w6 = d->w6;
    A.bop = (const TO *)d->bop;
    A.phi = (const TO *)phi;
    A.kv = (TO *)kv;
    A.done = done;
    return A;
}

template <class T, class TO>
ErowArgs<T, TO> erow_args(kfbi_domain *d, const void *uhat, void *ust, const int *done) {
    typedef typename Real<T>::type R;
    const bool low = sizeof(T) < sizeof(TO);
    ErowArgs<T, TO> A;
    A.M = d->M;
    A.n_rows = d->n_erows;
    A.erow_t = d->erow_t;
    A.erow_ptr = d->erow_ptr;
    A.erow_col = d->erow_col;
    A.uhat = (const T *)uhat;
    A.sine = low ? (const R *)d->sine32 : (const R *)d->sine;
    A.scu = low ? (const R *)d->scu32 : (const R *)d->scu;
    A.ust = (TO *)ust;
    A.done = done;
    return A;
}
template <class T, class TO>
size_t erow_lds(int M) {
    return (size_t)(2 * M + M / 2) * sizeof(typename Real<T>::type) + (size_t)kErowCols * sizeof(int32_t);
}
inline int erow_blocks(const kfbi_domain *d) { return (d->n_erows + kErowRows - 1) / kErowRows; }

// register slots per lane, M / 64 (one instantiation per grid size)
template <class F>
int erow_dispatch(int M, const F &f) {
    switch (M) {
        case 64: f.template go<1>(); break;
        case 128: f.template go<2>(); break;
        case 256: f.template go<4>(); break;
        case 512: f.template go<8>(); break;
        case 1024: f.template go<16>(); break;
        case 2048: f.template go<32>(); break;
        default:
            set_error("the row-wise stencil evaluation supports grids of 64 to 2048");
            return KFBI_ENOTSUP;
    }
    return KFBI_OK;
}

template <class T>
ExmArgs<T> exm_args(kfbi_domain *d, const void *ust, const void *phi, void *kv, const int *done) {
    return ExmArgs<T>{d->Nb, (const T *)ust, d->erow_nid, d->w6, (const T *)d->bop, (const T *)phi, (T *)kv, done};
}

template <class T, class TO>
EvalArgs<T, TO> eval_args(kfbi_domain *d, const void *uhat, void *out, const int *done) {
    typedef typename Real<T>::type R;
    const bool low = sizeof(T) < sizeof(TO);
    EvalArgs<T, TO> A;
    A.M = d->M;
    A.nnodes = 6 * d->Nb;
    A.node_stride = (int)(sizeof(Stencil) / sizeof(int32_t));
    A.nodes = reinterpret_cast<const int32_t *>(d->st);
    A.uhat = (const T *)uhat;
    A.sine = low ? (const R *)d->sine32 : (const R *)d->sine;
    A.scu = low ? (const R *)d->scu32 : (const R *)d->scu;
    A.out = (TO *)out;
    A.done = done;
    return A;
}

// launch shape of the tridiagonal kernel for one domain: modes per
// workgroup (the largest power of two <= 4 whose LDS tile stays within
// 32 KB, unless the domain fixes it; eight modes use 32-lane groups, fewer
// use 64), rows per lane, LDS and whether the sparse input is staged
struct TriShape {
    int mb, lanes, c, blocks;
    bool rows;                          // the register-row kernel
    size_t lds, lds_base, lds_stage;    // LDS in use; unstaged; staged
};

// the largest power of two <= 4 modes whose LDS tile stays within 32 KB
template <class T>
int tri_default_mb(int n) {
    int mb = 4;
    while (mb > 1 && (size_t)n * mb * sizeof(T) > 32768) mb >>= 1;
    return mb;
}

// rows: the register-row kernel, for sparse input with 1, 2 or 4 modes per
// workgroup and at least 4 rows per lane (tri_rows_ok)
template <class T>
TriShape tri_shape(const kfbi_domain *d, bool sparse, int mb_force = 0, bool rows = false) {
    TriShape S;
    const int n = d->M - 1;
    int mb = mb_force > 0 ? mb_force : d->tri_mb;
    if (mb <= 0) mb = tri_default_mb<T>(n);
    S.mb = mb;
    S.lanes = (mb == 8 && !rows) ? 32 : 64;
    S.c = 1;
    while (S.lanes * S.c < n) S.c <<= 1;
    S.blocks = (n + mb - 1) / mb;
    S.rows = rows;
    const size_t sine = (size_t)tri_sine_slots(d->M, rows) * sizeof(double);
    const size_t spart = sparse ? (size_t)d->n_seg * mb * sizeof(T) : 0;
    const size_t stage = sparse ? (size_t)d->n_irr * (sizeof(T) + sizeof(int32_t)) : 0;
    if (rows) {
        const size_t obuf = (size_t)std::min(S.c, 4) * 64 * (mb > 1 ? mb + 1 : 1) * sizeof(T);
        S.lds_base = sine + std::max(spart, obuf);
        S.lds_stage = sine + std::max(spart + stage, obuf);
    } else {
        S.lds_base = sine + ((size_t)n * mb + n / S.c + 1) * sizeof(T) + spart;
        S.lds_stage = S.lds_base + stage;
    }
    S.lds = S.lds_base;
    return S;
}

// whether the register-row kernel has an instantiation for this shape
inline bool tri_rows_ok(const TriShape &S) { return S.mb <= 8 && S.lanes == 64 && S.c >= 4 && S.c <= 32; }

}  // namespace

// The tridiagonal kernels the launch-shape timing may choose from: the
// environment variable KFBI_TRIDIAG_KERNEL = "tile" or "rows" restricts it to
// one of them (both compute the same values; for tests and diagnosis), -1
// when unset.
int tri_kernel_pref() {
    const char *v = std::getenv("KFBI_TRIDIAG_KERNEL");
    if (!v) return -1;
    if (std::strncmp(v, "tile", 4) == 0) return 0;
    if (std::strncmp(v, "rows", 4) == 0) return 1;
    return -1;
}

// "tile:<mb>" / "rows:<mb>" also fix the modes per workgroup; 0 when not
int tri_mb_pref() {
    const char *v = std::getenv("KFBI_TRIDIAG_KERNEL");
    if (!v || std::strlen(v) < 6 || v[4] != ':') return 0;
    const int mb = std::atoi(v + 5);
    return (mb == 1 || mb == 2 || mb == 4 || mb == 8) ? mb : 0;
}

// "<kernel>:<mb>:<s>" also fixes the staging of the sparse input (s = 0 or
// 1); -1 when not
int tri_stage_pref() {
    const char *v = std::getenv("KFBI_TRIDIAG_KERNEL");
    if (!v) return -1;
    const char *c = std::strchr(v, ':');
    if (!c) return -1;
    c = std::strchr(c + 1, ':');
    if (!c || (c[1] != '0' && c[1] != '1')) return -1;
    return c[1] - '0';
}

namespace {

template <class T>
TriArgs<T, typename High<T>::type> tri_args(kfbi_domain *d, const void *rhat, const void *corr, void *uhat,
                                            const int *done) {
    typedef typename High<T>::type TC;
    typedef typename Real<T>::type R;
    TriArgs<T, TC> A;
    A.M = d->M;
    A.h2 = d->h * d->h;
    A.rhat = (const T *)rhat;
    A.corr = (const TC *)corr;
    A.sp.irr_col = d->irr_col;
    A.sp.row_ptr = d->irr_row_ptr;
    A.sp.row_order = d->row_order;
    A.sp.seg_q0 = d->seg_q0;
    A.sp.seg_row = d->seg_row;
    A.sp.row_seg = d->row_seg;
    A.sp.seg_desc = d->seg_desc;
    A.sp.row_desc = d->row_desc;
    A.sp.row_span = d->row_span;
    A.sp.nnz = d->n_irr;
    A.sp.n_act = d->n_act_rows;
    A.sp.n_seg = d->n_seg;
    const bool low = sizeof(T) < sizeof(TC);
    A.sine = low ? (const R *)d->sine32 : (const R *)d->sine;
    A.etab = (const T *)(low ? d->etab32 : d->etab);
    A.elim = (const T *)(low ? d->elim32 : d->elim);
    A.tconv = low ? d->tconv32 : d->tconv;
    A.uhat = (T *)uhat;
    A.done = done;
    return A;
}

// one launch of a tridiagonal-kernel instantiation, single or batched
template <class T, class TC>
struct TriLaunchOne {
    TriArgs<T, TC> A;
    int blocks;
    size_t lds;
    hipStream_t s;
    template <int MB, int L, int C, bool ST>
    void go() const {
        k_tridiag<T, TC, MB, L, C, ST><<<blocks, MB * L, lds, s>>>(A);
    }
    template <int MB, int C, bool ST, bool DENSE>
    void go_rows() const {
        static_assert(!DENSE, "single-domain dense launches run the tile kernel");
        k_tridiag_rows<T, TC, MB, C, ST><<<blocks, MB * 64, lds, s>>>(A);
    }
};

template <class T, class TC, int MB, int LANES, int C, bool STAGE>
__global__ __launch_bounds__(MB *LANES) void kb_tridiag(const TriArgs<T, TC> *__restrict__ A,
                                                        const BlkMap *__restrict__ map) {
    const BlkMap e = map[xcd_tile(blockIdx.x, gridDim.x)];
    tridiag_body<T, TC, MB, LANES, C, STAGE>(A[e.inst], e.local);
}

template <class T, class TC, int MB, int C, bool STAGE, bool DENSE>
__global__ __launch_bounds__(MB * 64) void kb_tridiag_rows(const TriArgs<T, TC> *__restrict__ A,
                                                         const BlkMap *__restrict__ map) {
    const BlkMap e = map[xcd_tile(blockIdx.x, gridDim.x)];
    tridiag_rows_body<T, TC, MB, C, STAGE, DENSE>(A[e.inst], e.local);
}

template <class T, class TC>
struct TriLaunchBatch {
    const TriArgs<T, TC> *A;
    const BlkMap *map;
    int blocks;
    size_t lds;
    hipStream_t s;
    template <int MB, int L, int C, bool ST>
    void go() const {
        kb_tridiag<T, TC, MB, L, C, ST><<<blocks, MB * L, lds, s>>>(A, map);
    }
    template <int MB, int C, bool ST, bool DENSE>
    void go_rows() const {
        kb_tridiag_rows<T, TC, MB, C, ST, DENSE><<<blocks, MB * 64, lds, s>>>(A, map);
    }
};

template <class F>
void tri_dispatch(int mb, int c, bool stage, const F &f) {
#define KFBI_TRI(MBv, Lv, CC)                                  \
    do {                                                       \
        if (stage) f.template go<MBv, Lv, CC, true>();         \
        else f.template go<MBv, Lv, CC, false>();              \
    } while (0)
#define KFBI_TRI_C(MBv, Lv)                    \
    switch (c) {                               \
        case 1: KFBI_TRI(MBv, Lv, 1); break;   \
        case 2: KFBI_TRI(MBv, Lv, 2); break;   \
        case 4: KFBI_TRI(MBv, Lv, 4); break;   \
        case 8: KFBI_TRI(MBv, Lv, 8); break;   \
        case 16: KFBI_TRI(MBv, Lv, 16); break; \
        default: KFBI_TRI(MBv, Lv, 32); break; \
    }
    switch (mb) {
        case 8: KFBI_TRI_C(8, 32); break;
        case 4: KFBI_TRI_C(4, 64); break;
        case 2: KFBI_TRI_C(2, 64); break;
        default: KFBI_TRI_C(1, 64); break;
    }
#undef KFBI_TRI_C
#undef KFBI_TRI
}

// the register-row kernel: mb in {1, 2, 4, 8}, c in {4, ..., 32} (tri_rows_ok);
// WITH_DENSE: also the dense-input form (batched launches)
template <bool WITH_DENSE, class F>
void tri_rows_dispatch(int mb, int c, bool stage, bool dense, const F &f) {
#define KFBI_TRR(MBv, CC)                                                 \
    do {                                                                  \
        if constexpr (WITH_DENSE) {                                       \
            if (dense) {                                                  \
                if (stage) f.template go_rows<MBv, CC, true, true>();     \
                else f.template go_rows<MBv, CC, false, true>();          \
                break;                                                    \
            }                                                             \
        }                                                                 \
        if (stage) f.template go_rows<MBv, CC, true, false>();            \
        else f.template go_rows<MBv, CC, false, false>();                 \
    } while (0)
#define KFBI_TRR_C(MBv)                       \
    switch (c) {                              \
        case 4: KFBI_TRR(MBv, 4); break;      \
        case 8: KFBI_TRR(MBv, 8); break;      \
        case 16: KFBI_TRR(MBv, 16); break;    \
        default: KFBI_TRR(MBv, 32); break;    \
    }
    switch (mb) {
        case 8: KFBI_TRR_C(8); break;
        case 4: KFBI_TRR_C(4); break;
        case 2: KFBI_TRR_C(2); break;
        default: KFBI_TRR_C(1); break;
    }
#undef KFBI_TRR_C
#undef KFBI_TRR
}

// a tile- or row-kernel launch of shape S
template <class F>
void tri_launch(const TriShape &S, bool stage, const F &f) {
    if (S.rows) tri_rows_dispatch<false>(S.mb, S.c, stage, false, f);
    else tri_dispatch(S.mb, S.c, stage, f);
}

template <class T>
int launch_tridiag(kfbi_domain *d, const void *rhat, const void *corr, void *uhat, const int *done) {
    typedef typename High<T>::type TC;
    const int n = d->M - 1;
    // sparse input: the row kernel when timing chose it.  Dense input runs
    // the tile kernel, at the timed modes per workgroup unless those are 8
    // (a row-kernel choice: the tile kernel's 8-mode shape has 32-lane groups
    // and other values), then at its default
    const bool rows = corr && !rhat && d->tri_rows;
    const int mb_tile = (d->tri_rows && d->tri_mb == 8) ? tri_default_mb<T>(n) : 0;
    TriShape S = tri_shape<T>(d, corr != nullptr, rows ? 0 : mb_tile, rows);
    if (S.rows && !tri_rows_ok(S)) S = tri_shape<T>(d, corr != nullptr, mb_tile);
    if (S.c > 32 || S.lds > kTriLdsMax) {
        set_error("grid too large for the tridiagonal kernel");
        return KFBI_ENOTSUP;
    }
    // stage the sparse right-hand side in LDS when it fits (unless timing
    // found the unstaged kernel faster)
    const bool stage = corr && S.lds_stage <= kTriLdsMax && d->tri_stage != 0;
    if (stage) S.lds = S.lds_stage;
    TriLaunchOne<T, TC> L{tri_args<T>(d, rhat, corr, uhat, done), S.blocks, S.lds, d->stream};
    const int ps = prof_begin(d);
    tri_launch(S, stage, L);
    KFBI_CHECK_LAUNCH();
    {
        // algorithmic bytes: write U^ (and read R^ when dense) plus the sparse input
        const double es = sizeof(T), nn = (double)n * n;
        const double sparse = corr ? (double)d->n_irr * (es + 4.0) + 4.0 * (n + 1) : 0.0;
        prof_end(d, ps, rhat ? KFBI_K_TRIDIAG_DENSE : KFBI_K_TRIDIAG_SPARSE,
                 es * nn * (rhat ? 2.0 : 1.0) + sparse);
    }
    return KFBI_OK;
}

}  // namespace

// Times the sparse-input tridiagonal launch of this domain for 1, 2 and 4
// modes per workgroup (64-lane mode groups: the same operations in the same
// order for every mode), with and without LDS staging, in the tile and the
// register-row kernels, on the domain's own tables, and keeps the fastest.
// Each shape is timed in three rounds over all shapes (20 launches each,
// after one untimed) and scored by its best round, so that a clock ramp or
// a transient on the device does not decide the choice.  Writes only the
// scratch transforms.
template <class T>
int tune_tridiag_t(kfbi_domain *d) {
    typedef typename High<T>::type TC;
    hipStream_t s = d->stream;
    KFBI_HIP(hipMemsetAsync(d->corr, 0, (size_t)d->n_irr * sizeof(TC), s));
    struct Cand {
        int rows, mb, stage;
        TriShape S;
        float best;
    };
    std::vector<Cand> cands;
    const int pref = tri_kernel_pref();
    for (int rows : {0, 1}) {
        if (pref >= 0 && rows != pref) continue;
        for (int mb : {1, 2, 4, 8}) {
            if (mb == 8 && !rows) continue;  // the tile kernel's 8-mode shape has 32-lane groups
            if (tri_mb_pref() > 0 && mb != tri_mb_pref()) continue;
            const TriShape S = tri_shape<T>(d, true, mb, rows != 0);
            if (S.c > 32 || S.lds > kTriLdsMax || (rows && !tri_rows_ok(S))) continue;
            for (int stage : {0, 1}) {
                if (stage && S.lds_stage > kTriLdsMax) continue;
                if (tri_stage_pref() >= 0 && stage != tri_stage_pref()) continue;
                cands.push_back(Cand{rows, mb, stage, S, 1e30f});
            }
        }
    }
    if (cands.empty()) return KFBI_OK;  // the default shape stays
    hipEvent_t e0 = nullptr, e1 = nullptr;
    KFBI_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        set_error("hipEventCreate failed");
        return KFBI_EDEVICE;
    }
    int st = KFBI_OK;
    for (int round = 0; round < 3 && st == KFBI_OK; ++round) {
        for (Cand &c : cands) {
            const size_t lds = c.stage ? c.S.lds_stage : c.S.lds;
            TriLaunchOne<T, TC> L{tri_args<T>(d, nullptr, d->corr, d->uhat, nullptr), c.S.blocks, lds, s};
            tri_launch(c.S, c.stage != 0, L);
            if (hipEventRecord(e0, s) != hipSuccess) st = KFBI_EDEVICE;
            for (int r = 0; r < 20; ++r) tri_launch(c.S, c.stage != 0, L);
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) st = KFBI_EDEVICE;
            float ms = 0.f;
            if (st == KFBI_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = KFBI_EDEVICE;
            if (st != KFBI_OK) break;
            c.best = std::min(c.best, ms);
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (st != KFBI_OK) {
        set_error("timing the tridiagonal launch shapes failed");
        return st;
    }
    const Cand *win = &cands[0];
    for (const Cand &c : cands)
        if (c.best < win->best) win = &c;
    d->tri_mb = win->mb;
    d->tri_stage = win->stage ? -1 : 0;
    d->tri_rows = win->rows;
    return KFBI_OK;
}

int tune_tridiag(kfbi_domain *d) {
    if (d->tri_tuned) return KFBI_OK;
    d->tri_tuned = true;
    if (d->tri_mb > 0) return KFBI_OK;
    return d->cplx ? tune_tridiag_t<cd>(d) : tune_tridiag_t<double>(d);
}

int ensure_coefficients(kfbi_domain *d, double kre, double kim) {
    if (d->coef_valid && d->coef_kre == kre && d->coef_kim == kim) return KFBI_OK;
    const int M = d->M, n = M - 1;
    const double h2 = d->h * d->h;
    if (d->cplx)
        k_coef<cd><<<(n + 127) / 128, 128, 0, d->stream>>>(M, kre * h2, kim * h2, (cd *)d->etab,
                                                          (cd *)d->elim, d->tconv);
    else
        k_coef<double><<<(n + 127) / 128, 128, 0, d->stream>>>(M, kre * h2, 0.0, (double *)d->etab,
                                                              (double *)d->elim, d->tconv);
    KFBI_CHECK_LAUNCH();
    d->coef_valid = true;
    d->coef_kre = kre;
    d->coef_kim = kim;
    return KFBI_OK;
}

namespace {
__global__ void k_sine32(int M, float *s, float *scu) {
    int m = blockIdx.x * blockDim.x + threadIdx.x;
    // a period and its first quarter again (2M + M/2 entries)
    if (m < 2 * M + M / 2) s[m] = (float)sinpi_sym(m, M);
    if (m < max(1, M / 32)) {
        scu[2 * m] = (float)sinpi_sym(64 * m, M);
        scu[2 * m + 1] = (float)sinpi_sym(64 * m + M / 2, M);
    }
}
}  // namespace

size_t low_tables_bytes_pending(const kfbi_domain *d) {
    if (d->uhat32) return 0;
    const size_t M = (size_t)d->M, n = M - 1, ls = d->cplx ? sizeof(cf) : sizeof(float);
    return 2 * n * n * ls + n * ls + n * sizeof(int32_t) + (2 * M + M / 2) * sizeof(float) +
           2 * (size_t)std::max(1, d->M / 32) * sizeof(float);
}

// FP32 / complex64 coefficient table and scratch for the mixed-precision
// grid solve (allocated on first use)
int ensure_coefficients_low(kfbi_domain *d, double kre, double kim) {
    if (d->coef32_valid && d->coef32_kre == kre && d->coef32_kim == kim) return KFBI_OK;
    const int M = d->M, n = M - 1;
    const size_t ls = d->cplx ? sizeof(cf) : sizeof(float);
    if (!d->uhat32) {
        KFBI_TRY(dalloc(d, &d->uhat32, (size_t)n * n * ls));
        KFBI_TRY(dalloc(d, &d->etab32, (size_t)n * n * ls));
        KFBI_TRY(dalloc(d, &d->elim32, (size_t)n * ls));
        KFBI_TRY(dalloc(d, (void **)&d->tconv32, (size_t)n * sizeof(int32_t)));
        KFBI_TRY(dalloc(d, (void **)&d->sine32, (size_t)(2 * M + M / 2) * sizeof(float)));
        KFBI_TRY(dalloc(d, (void **)&d->scu32, (size_t)2 * std::max(1, M / 32) * sizeof(float)));
        k_sine32<<<(2 * M + M / 2 + 255) / 256, 256, 0, d->stream>>>(M, d->sine32, d->scu32);
        KFBI_CHECK_LAUNCH();
    }
    const double h2 = d->h * d->h;
    if (d->cplx)
        k_coef<cf><<<(n + 127) / 128, 128, 0, d->stream>>>(M, kre * h2, kim * h2, (cf *)d->etab32,
                                                          (cf *)d->elim32, d->tconv32);
    else
        k_coef<float><<<(n + 127) / 128, 128, 0, d->stream>>>(M, kre * h2, 0.0, (float *)d->etab32,
                                                             (float *)d->elim32, d->tconv32);
    KFBI_CHECK_LAUNCH();
    d->coef32_valid = true;
    d->coef32_kre = kre;
    d->coef32_kim = kim;
    return KFBI_OK;
}

int tridiag_solve_phi(kfbi_domain *d, const void *phi, void *uhat_out, const int *done, bool low) {
    if (!d->op_merged) {
        set_error("the density form of the grid solve needs the merged correction operator");
        return KFBI_ENOTSUP;
    }
    // corrections once, by many workgroups (every tridiagonal workgroup
    // needs all of them), then the sparse grid solve
    KFBI_TRY(corrections_of_density(d, phi, d->corr, done));
    if (low) {
        if (d->cplx) return launch_tridiag<cf>(d, nullptr, d->corr, uhat_out, done);
        return launch_tridiag<float>(d, nullptr, d->corr, uhat_out, done);
    }
    if (d->cplx) return launch_tridiag<cd>(d, nullptr, d->corr, uhat_out, done);
    return launch_tridiag<double>(d, nullptr, d->corr, uhat_out, done);
}


int tridiag_solve_low(kfbi_domain *d, const void *corr, void *uhat32_out, const int *done) {
    if (d->cplx) return launch_tridiag<cf>(d, nullptr, corr, uhat32_out, done);
    return launch_tridiag<float>(d, nullptr, corr, uhat32_out, done);
}

int dst_rows_dense(kfbi_domain *d, const void *grid, bool mask_inside, void *rhat_out) {
    const uint8_t *mask = mask_inside ? d->flags : nullptr;
    if (d->cplx) return launch_dst<cd>(d, grid, true, mask, rhat_out, false, 1.0);
    return launch_dst<double>(d, grid, true, mask, rhat_out, false, 1.0);
}

// the b-solve's forward DST of f (masked to the inside) and the
// corrections of f alone (no density), in one launch
int dst_rows_dense_corr(kfbi_domain *d, const void *grid, void *rhat_out, double kre, double kim,
                        const void *f_gamma, void *corr_out) {
    alignas(16) unsigned char buf[sizeof(CorrArgs<cd>)];
    batch_fill_corr(d, kre, kim, nullptr, f_gamma, corr_out, nullptr, buf);
    const int M = d->M, n = M - 1;
    const int ps = prof_begin(d);
    if (d->cplx) {
        const int nd = dst_blocks<cd>(M);
        k_dst_rows_corr<cd><<<nd + (d->n_irr + 255) / 256, 256, dst_lds(M), d->stream>>>(
            dst_args<cd>(d, grid, true, d->flags, rhat_out, false, 1.0, nullptr), *(const CorrArgs<cd> *)buf, nd);
    } else {
        const int nd = dst_blocks<double>(M);
        k_dst_rows_corr<double><<<nd + (d->n_irr + 255) / 256, 256, dst_lds(M), d->stream>>>(
            dst_args<double>(d, grid, true, d->flags, rhat_out, false, 1.0, nullptr),
            *(const CorrArgs<double> *)buf, nd);
    }
    KFBI_CHECK_LAUNCH();
    const double es = elem_size(d), nn = (double)n * n;
    prof_end(d, ps, KFBI_K_DST, es * (nn + nn) + nn + (double)d->n_irr * (sizeof(IrrNode) + es));
    return KFBI_OK;
}

int idst_rows_dense(kfbi_domain *d, const void *uhat, void *grid_out) {
    return idst_rows_dense_ctl(d, uhat, grid_out, nullptr);
}

int idst_rows_dense_ctl(kfbi_domain *d, const void *uhat, void *grid_out, const int *done, const GridUpdate *up) {
    double scale = 2.0 / d->M;
    if (d->cplx) return launch_dst<cd>(d, uhat, false, nullptr, grid_out, true, scale, done, up);
    return launch_dst<double>(d, uhat, false, nullptr, grid_out, true, scale, done, up);
}

int tridiag_solve(kfbi_domain *d, const void *rhat, const void *corr, void *uhat_out) {
    return tridiag_solve_ctl(d, rhat, corr, uhat_out, nullptr);
}

int tridiag_solve_ctl(kfbi_domain *d, const void *rhat, const void *corr, void *uhat_out, const int *done) {
    if (d->cplx) return launch_tridiag<cd>(d, rhat, corr, uhat_out, done);
    return launch_tridiag<double>(d, rhat, corr, uhat_out, done);
}

int eval_stencil_nodes(kfbi_domain *d, const void *uhat, void *ust_out) {
    return eval_stencil_nodes_ctl(d, uhat, ust_out, nullptr, false);
}



int corrections_of_density(kfbi_domain *d, const void *phi, void *corr_out, const int *done, const void *base,
                           void *copy_out) {
    const int nnz = d->n_irr;
    const int blocks = (nnz + 63) / 64 + (copy_out ? (d->Nb + 63) / 64 : 0);
    const int ps = prof_begin(d);
    if (d->cplx)
        k_corr_phi<cd><<<blocks, 64, 0, d->stream>>>(corr_phi_args<cd>(d, phi, corr_out, done, base, copy_out));
    else
        k_corr_phi<double><<<blocks, 64, 0, d->stream>>>(
            corr_phi_args<double>(d, phi, corr_out, done, base, copy_out));
    KFBI_CHECK_LAUNCH();
    const double es = elem_size(d);
    prof_end(d, ps, KFBI_K_CORRECTIONS, (double)nnz * (kCorrWin * es + 4.0 + es) + (double)d->Nb * es);
    return KFBI_OK;
}

int eval_extract_ctl(kfbi_domain *d, const void *uhat, const void *phi, void *kv_out, const int *done, bool low) {
    const int Nb = d->Nb;
    const int ps = prof_begin(d);
    if (d->cplx) {
        if (low) evx_dispatch(d->M, EvxLaunch<cf, cd>{evx_args<cf, cd>(d, uhat, phi, kv_out, done), Nb, d->stream});
        else evx_dispatch(d->M, EvxLaunch<cd, cd>{evx_args<cd, cd>(d, uhat, phi, kv_out, done), Nb, d->stream});
    } else {
        if (low)
            evx_dispatch(d->M, EvxLaunch<float, double>{evx_args<float, double>(d, uhat, phi, kv_out, done), Nb,
                                                        d->stream});
        else
            evx_dispatch(d->M, EvxLaunch<double, double>{evx_args<double, double>(d, uhat, phi, kv_out, done), Nb,
                                                         d->stream});
    }
    KFBI_CHECK_LAUNCH();
    const double es = low ? elem_size(d) / 2.0 : elem_size(d), eo = elem_size(d);
    prof_end(d, ps, KFBI_K_EVAL_NODES,
             (double)Nb * (6.0 * ((d->M - 1) * es + 4.0) + 6.0 * 8.0 + 5.0 * eo + 2.0 * eo));
    return KFBI_OK;
}

int eval_stencil_nodes_ctl(kfbi_domain *d, const void *uhat, void *ust_out, const int *done, bool low) {
    const int nn = 6 * d->Nb;
    const int grid = (nn + 3) / 4;
    const int ps = prof_begin(d);
    if (d->cplx) {
        if (low) k_eval_nodes<cf, cd><<<grid, 256, 0, d->stream>>>(eval_args<cf, cd>(d, uhat, ust_out, done));
        else k_eval_nodes<cd, cd><<<grid, 256, 0, d->stream>>>(eval_args<cd, cd>(d, uhat, ust_out, done));
    } else {
        if (low)
            k_eval_nodes<float, double><<<grid, 256, 0, d->stream>>>(
                eval_args<float, double>(d, uhat, ust_out, done));
        else
            k_eval_nodes<double, double><<<grid, 256, 0, d->stream>>>(
                eval_args<double, double>(d, uhat, ust_out, done));
    }
    KFBI_CHECK_LAUNCH();
    const double es = low ? elem_size(d) / 2.0 : elem_size(d);
    prof_end(d, ps, KFBI_K_EVAL_NODES, (double)nn * ((d->M - 1) * es + 4.0 + elem_size(d)));
    return KFBI_OK;
}

// The b-solve's stencil values and extraction, out = g + scale U+ with the
// jumps of f alone (no density), in one launch (k_eval_extract_gen)
int eval_extract_boundary(kfbi_domain *d, double kre, double kim, const void *uhat, const void *f_gamma,
                          const void *g, double scale, void *out) {
    alignas(16) unsigned char buf[sizeof(ExtArgs<cd>)];
    batch_fill_ext(d, kre, kim, nullptr, nullptr, f_gamma, g, scale, out, nullptr, buf);
    const int Nb = d->Nb;
    const int ps = prof_begin(d);
    if (d->cplx) {
        ExtArgs<cd> X = *(const ExtArgs<cd> *)buf;
        X.nid = nullptr;
        evx_dispatch(d->M, EvxGenLaunch<cd>{eval_args<cd, cd>(d, uhat, nullptr, nullptr), X, Nb, d->stream});
    } else {
        ExtArgs<double> X = *(const ExtArgs<double> *)buf;
        X.nid = nullptr;
        evx_dispatch(d->M, EvxGenLaunch<double>{eval_args<double, double>(d, uhat, nullptr, nullptr), X, Nb,
                                                d->stream});
    }
    KFBI_CHECK_LAUNCH();
    const double es = elem_size(d);
    prof_end(d, ps, KFBI_K_EXTRACT,
             (double)Nb * (6.0 * ((d->M - 1) * es + 4.0) + sizeof(Colloc) + sizeof(Stencil) + 3.0 * es));
    return KFBI_OK;
}

// ---------------------------------------------------------------------------
// Batched launches: one grid runs the blocks of many instances; workgroup b
// looks up (instance, local block) in a map and reads that instance's
// argument block.  The instances of a launch share one scalar type: real
// (FP64, FP32 inner solves) or complex (complex128, complex64 inner solves).
// ---------------------------------------------------------------------------
namespace {
template <class T>
__global__ __launch_bounds__(256) void kb_dst_rows(const DstArgs<T> *__restrict__ A, const BlkMap *__restrict__ map) {
    const BlkMap e = map[blockIdx.x];
    dst_rows_body(A[e.inst], e.local);
}
template <class T>
__global__ __launch_bounds__(256) void kb_zero_edge_rows(const ZeroArgs<T> *__restrict__ A,
                                                         const BlkMap *__restrict__ map) {
    const BlkMap e = map[blockIdx.x];
    zero_edge_body(A[e.inst], e.local);
}
template <class T, class TO>
__global__ __launch_bounds__(256) void kb_eval_nodes(const EvalArgs<T, TO> *__restrict__ A,
                                                     const BlkMap *__restrict__ map) {
    const BlkMap e = map[blockIdx.x];
    eval_nodes_body(A[e.inst], e.local);
}
template <class T, class TO>
__global__ __launch_bounds__(384) void kb_eval_extract(const EvxArgs<T, TO> *__restrict__ A,
                                                       const BlkMap *__restrict__ map) {
    const BlkMap e = map[blockIdx.x];
    eval_extract_body<T, TO, 0>(A[e.inst], e.local);  // members of any M
}
template <class TC>
__global__ __launch_bounds__(64) void kb_corr_phi(const CorrPhiArgs<TC> *__restrict__ A,
                                                  const BlkMap *__restrict__ map) {
    const BlkMap e = map[blockIdx.x];
    corr_phi_body(A[e.inst], e.local);
}
template <class T, class TO>
struct ErowLaunchBatch {
    const ErowArgs<T, TO> *A;
    const BlkMap *map;
    int blocks;
    size_t lds;
    hipStream_t s;
    template <int KR>
    void go() const;
};
template <class T, class TO, int KR>
__global__ __launch_bounds__(256) void kb_eval_rows(const ErowArgs<T, TO> *__restrict__ A,
                                                    const BlkMap *__restrict__ map) {
    const BlkMap e = map[blockIdx.x];
    eval_rows_body<T, TO, KR>(A[e.inst], e.local);
}
template <class T, class TO>
template <int KR>
void ErowLaunchBatch<T, TO>::go() const {
    kb_eval_rows<T, TO, KR><<<blocks, 256, lds, s>>>(A, map);
}
template <class T>
__global__ __launch_bounds__(256) void kb_extract_merged(const ExmArgs<T> *__restrict__ A,
                                                         const BlkMap *__restrict__ map) {
    const BlkMap e = map[blockIdx.x];
    extract_merged_body(A[e.inst], e.local);
}
}  // namespace

// argument blocks of one member, written to host memory: a batched kernel
// indexes its blocks with the size of its own instantiation, so the stride is
// the exact size for the batch's scalar type
namespace {
template <class R, class C>
size_t args_size(bool cplx) {
    return cplx ? sizeof(C) : sizeof(R);
}
}  // namespace

size_t batch_args_size(int kind, bool cplx) {
    switch (kind) {
        case kBaDst: return args_size<DstArgs<double>, DstArgs<cd>>(cplx);
        case kBaZero: return args_size<ZeroArgs<double>, ZeroArgs<cd>>(cplx);
        case kBaTri64: return args_size<TriArgs<double, double>, TriArgs<cd, cd>>(cplx);
        case kBaTri32: return args_size<TriArgs<float, double>, TriArgs<cf, cd>>(cplx);
        case kBaEval: return args_size<EvalArgs<double, double>, EvalArgs<cd, cd>>(cplx);
        case kBaEvx64: return args_size<EvxArgs<double, double>, EvxArgs<cd, cd>>(cplx);
        case kBaEvx32: return args_size<EvxArgs<float, double>, EvxArgs<cf, cd>>(cplx);
        case kBaCorrPhi: return args_size<CorrPhiArgs<double>, CorrPhiArgs<cd>>(cplx);
        case kBaErow64: return args_size<ErowArgs<double, double>, ErowArgs<cd, cd>>(cplx);
        case kBaErow32: return args_size<ErowArgs<float, double>, ErowArgs<cf, cd>>(cplx);
        case kBaExm: return args_size<ExmArgs<double>, ExmArgs<cd>>(cplx);
        default: return 0;
    }
}

void batch_fill_dst(kfbi_domain *d, const void *in, bool in_grid, bool mask_inside, void *out, bool out_grid,
                    double scale, const int *done, void *dst) {
    const uint8_t *mask = mask_inside ? d->flags : nullptr;
    if (d->cplx) *(DstArgs<cd> *)dst = dst_args<cd>(d, in, in_grid, mask, out, out_grid, scale, done);
    else *(DstArgs<double> *)dst = dst_args<double>(d, in, in_grid, mask, out, out_grid, scale, done);
}
void batch_fill_zero(kfbi_domain *d, void *grid, const int *done, void *dst) {
    if (d->cplx) *(ZeroArgs<cd> *)dst = ZeroArgs<cd>{d->M, (cd *)grid, done};
    else *(ZeroArgs<double> *)dst = ZeroArgs<double>{d->M, (double *)grid, done};
}
void batch_fill_tri(kfbi_domain *d, const void *rhat, const void *corr, void *uhat, const int *done, bool low,
                    void *dst) {
    if (d->cplx) {
        if (low) *(TriArgs<cf, cd> *)dst = tri_args<cf>(d, rhat, corr, uhat, done);
        else *(TriArgs<cd, cd> *)dst = tri_args<cd>(d, rhat, corr, uhat, done);
    } else {
        if (low) *(TriArgs<float, double> *)dst = tri_args<float>(d, rhat, corr, uhat, done);
        else *(TriArgs<double, double> *)dst = tri_args<double>(d, rhat, corr, uhat, done);
    }
}
void batch_fill_eval(kfbi_domain *d, const void *uhat, void *out, const int *done, void *dst) {
    if (d->cplx) *(EvalArgs<cd, cd> *)dst = eval_args<cd, cd>(d, uhat, out, done);
    else *(EvalArgs<double, double> *)dst = eval_args<double, double>(d, uhat, out, done);
}
void batch_fill_evx(kfbi_domain *d, const void *uhat, const void *phi, void *kv, const int *done, bool low,
                    void *dst) {
    if (d->cplx) {
        if (low) *(EvxArgs<cf, cd> *)dst = evx_args<cf, cd>(d, uhat, phi, kv, done);
        else *(EvxArgs<cd, cd> *)dst = evx_args<cd, cd>(d, uhat, phi, kv, done);
    } else {
        if (low) *(EvxArgs<float, double> *)dst = evx_args<float, double>(d, uhat, phi, kv, done);
        else *(EvxArgs<double, double> *)dst = evx_args<double, double>(d, uhat, phi, kv, done);
    }
}
void batch_fill_corr_phi(kfbi_domain *d, const void *phi, void *corr, const int *done, void *dst,
                         const void *base) {
    if (d->cplx) *(CorrPhiArgs<cd> *)dst = corr_phi_args<cd>(d, phi, corr, done, base);
    else *(CorrPhiArgs<double> *)dst = corr_phi_args<double>(d, phi, corr, done, base);
}
void batch_fill_erow(kfbi_domain *d, const void *uhat, void *ust, const int *done, bool low, void *dst) {
    if (d->cplx) {
        if (low) *(ErowArgs<cf, cd> *)dst = erow_args<cf, cd>(d, uhat, ust, done);
        else *(ErowArgs<cd, cd> *)dst = erow_args<cd, cd>(d, uhat, ust, done);
    } else {
        if (low) *(ErowArgs<float, double> *)dst = erow_args<float, double>(d, uhat, ust, done);
        else *(ErowArgs<double, double> *)dst = erow_args<double, double>(d, uhat, ust, done);
    }
}
void batch_fill_exm(kfbi_domain *d, const void *ust, const void *phi, void *kv, const int *done, void *dst) {
    if (d->cplx) *(ExmArgs<cd> *)dst = exm_args<cd>(d, ust, phi, kv, done);
    else *(ExmArgs<double> *)dst = exm_args<double>(d, ust, phi, kv, done);
}

int batch_blocks(const kfbi_domain *d, int kind) {
    switch (kind) {
        case kBaDst: return d->cplx ? dst_blocks<cd>(d->M) : dst_blocks<double>(d->M);
        case kBaZero: return (d->M + 1 + 255) / 256;
        case kBaTri64: return d->cplx ? tri_shape<cd>(d, true).blocks : tri_shape<double>(d, true).blocks;
        case kBaTri32: return d->cplx ? tri_shape<cf>(d, true).blocks : tri_shape<float>(d, true).blocks;
        case kBaEval: return (6 * d->Nb + 3) / 4;
        case kBaEvx64:
        case kBaEvx32: return d->Nb;
        case kBaCorrPhi: return (d->n_irr + 63) / 64;
        case kBaErow64:
        case kBaErow32: return erow_blocks(d);
        case kBaExm: return (d->Nb + 255) / 256;
        default: return 0;
    }
}

// launch shape of the tridiagonal kernel shared by a batch class (equal M,
// mb and c; LDS the largest over the members; staged when all fit)
int batch_tri_shape(kfbi_domain *const *doms, int n, bool sparse, bool low, BatchTriShape *out, int mb, int stage_pref,
                    bool rows) {
    const bool cplx = doms[0]->cplx;
    // the static default, not a member's own timed choice, when none is given
    if (mb <= 0) {
        const int n0 = doms[0]->M - 1;
        mb = cplx ? (low ? tri_default_mb<cf>(n0) : tri_default_mb<cd>(n0))
                  : (low ? tri_default_mb<float>(n0) : tri_default_mb<double>(n0));
    }

    for (int q = 0; q < n; ++q) {
        kfbi_domain *d = doms[q];
        const TriShape S = cplx ? (low ? tri_shape<cf>(d, sparse, mb, rows) : tri_shape<cd>(d, sparse, mb, rows))
                                : (low ? tri_shape<float>(d, sparse, mb, rows) : tri_shape<double>(d, sparse, mb, rows));
        if (rows && !tri_rows_ok(S)) {
            set_error("no register-row tridiagonal kernel for this shape");
            return KFBI_ENOTSUP;
        }
        if (q == 0) {
            out->mb = S.mb;
            out->c = S.c;
            out->rows = rows;
            out->dense = false;
            out->lds = S.lds_base;
            out->stage_lds = S.lds_stage;
        } else {
            if (S.mb != out->mb || S.c != out->c) {
                set_error("batch class members differ in tridiagonal launch shape");
                return KFBI_EINVAL;
            }
            out->lds = std::max(out->lds, S.lds_base);
            out->stage_lds = std::max(out->stage_lds, S.lds_stage);
        }
    }
    if (out->c > 32 || out->lds > kTriLdsMax) {
        set_error("grid too large for the tridiagonal kernel");
        return KFBI_ENOTSUP;
    }
    out->stage = sparse && out->stage_lds <= kTriLdsMax && stage_pref != 0;
    if (stage_pref == 1 && !out->stage) {
        set_error("staged sparse input does not fit");
        return KFBI_ENOTSUP;
    }
    if (out->stage) out->lds = out->stage_lds;
    out->blocks_per = 0;
    return KFBI_OK;
}

int batch_tri_blocks(const kfbi_domain *d, int mb) {
    return (d->M - 1 + mb - 1) / mb;
}

namespace {
// one batched launch of kind `kind` with element type T (double or cd) and
// inner-solve type TL (float or cf)
template <class T, class TL>
int batch_launch_t(int kind, const void *args, const BlkMap *map, int blocks, int M, const BatchTriShape *shape,
                   hipStream_t s) {
    switch (kind) {
        case kBaDst:
            kb_dst_rows<T><<<blocks, 256, dst_lds(M), s>>>((const DstArgs<T> *)args, map);
            break;
        case kBaZero:
            kb_zero_edge_rows<T><<<blocks, 256, 0, s>>>((const ZeroArgs<T> *)args, map);
            break;
        case kBaTri64: {
            TriLaunchBatch<T, T> L{(const TriArgs<T, T> *)args, map, blocks, shape->lds, s};
            if (shape->rows) tri_rows_dispatch<true>(shape->mb, shape->c, shape->stage, shape->dense, L);
            else tri_dispatch(shape->mb, shape->c, shape->stage, L);
            break;
        }
        case kBaTri32: {
            TriLaunchBatch<TL, T> L{(const TriArgs<TL, T> *)args, map, blocks, shape->lds, s};
            if (shape->rows) tri_rows_dispatch<false>(shape->mb, shape->c, shape->stage, false, L);
            else tri_dispatch(shape->mb, shape->c, shape->stage, L);
            break;
        }
        case kBaEval:
            kb_eval_nodes<T, T><<<blocks, 256, 0, s>>>((const EvalArgs<T, T> *)args, map);
            break;
        case kBaEvx64:
            kb_eval_extract<T, T><<<blocks, 384, 0, s>>>((const EvxArgs<T, T> *)args, map);
            break;
        case kBaEvx32:
            kb_eval_extract<TL, T><<<blocks, 384, 0, s>>>((const EvxArgs<TL, T> *)args, map);
            break;
        case kBaCorrPhi:
            kb_corr_phi<T><<<blocks, 64, 0, s>>>((const CorrPhiArgs<T> *)args, map);
            break;
        case kBaErow64: {
            ErowLaunchBatch<T, T> L{(const ErowArgs<T, T> *)args, map, blocks, erow_lds<T, T>(M), s};
            KFBI_TRY(erow_dispatch(M, L));
            break;
        }
        case kBaErow32: {
            ErowLaunchBatch<TL, T> L{(const ErowArgs<TL, T> *)args, map, blocks, erow_lds<TL, T>(M), s};
            KFBI_TRY(erow_dispatch(M, L));
            break;
        }
        case kBaExm:
            kb_extract_merged<T><<<blocks, 256, 0, s>>>((const ExmArgs<T> *)args, map);
            break;
        default:
            set_error("unknown batched kernel");
            return KFBI_EINVAL;
    }
    KFBI_CHECK_LAUNCH();
    return KFBI_OK;
}
}  // namespace

int batch_launch(int kind, const void *args, const BlkMap *map, int blocks, int M, const BatchTriShape *shape,
                 hipStream_t s, bool cplx) {
    if (blocks <= 0) return KFBI_OK;
    if (cplx) return batch_launch_t<cd, cf>(kind, args, map, blocks, M, shape, s);
    return batch_launch_t<double, float>(kind, args, map, blocks, M, shape, s);
}

}  // namespace kfbi
