// GMRES for the discrete second-kind integral equation (3.17) on the device.
//
// The paper iterates (3.17) with Richardson's method (3.21) and names GMRES
// as the better Krylov choice in its conclusion; this library uses
// restarted GMRES(m).  All Krylov state lives on the device: a control block
// (current column j, iteration count, residual, done flag), the basis V,
// the Hessenberg matrix H and the Givens rotations.  Every kernel of an
// iteration reads j and the done flag from the control block, so a chunk of
// iterations is enqueued without host round trips and the host reads the
// control block once per chunk; after convergence the remaining kernels of
// the chunk return at once.
//
// Arnoldi orthogonalisation is classical Gram-Schmidt applied twice (CGS2:
// two passes of all inner products at once, so a step costs a fixed handful
// of workgroup reductions instead of one per basis vector); it gives the same
// basis as modified Gram-Schmidt up to rounding.  (A conditional second pass
// does not pay here: for the second-kind operator 1/2 I + W the projection
// removes most of K v_j, so the reorthogonalisation test nearly always fires.)
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <string>
#include <cstring>
#include <vector>

#include "kfbi_internal.h"

namespace kfbi {

// eta > 0 (mixed precision): a cycle runs until its residual estimate falls
// below thresh = max(tol ||b||, eta beta); convergence is then decided only
// by the FP64 residual computed at the start of the next cycle
//
// Device-driven schedule (merged-operator path): the solve is a sequence of
// identical slots, each one grid solve followed by one control kernel that
// acts on `state`: a cycle start (r = b - K x, stop test, v_0), an Arnoldi
// step, or nothing once finished.  The control kernel sets the gate words
// read by the next slot's grid-solve kernels (skip64 / skip32: FP64 / FP32
// solve not needed) and by the final solve enqueued after the slots
// (skip_tail, cleared when finished).
constexpr int kStIter = 0, kStStart = 1, kStDone = 2;

struct GmCtl {
    int j, done, iters, converged;
    int max_iter, m, fixed, breakdown;
    double tol, bnorm, beta, resid;
    double eta, thresh;
    int state, skip64, skip32, skip_tail;
    int slot, cycles, mixed, pad;
};

// host-visible copy of the control block's outcome, in pinned host memory;
// written by every control kernel, seq last.  seq carries the publishing
// slot and its state, 4 slot + state, so that the host reads both in one
// load; the other fields were complete before that store, and after a
// publish with state Done nothing is published until the next solve resets
// seq, so a host that has read Done from seq reads final fields.
struct GmMirror {
    int seq, state, iters, converged, cycles, pad;
    double resid, bnorm;
};

// the slot count and state a mirror's seq word holds (host side)
inline void mirror_seq(const GmMirror *mh, int *slot, int *state) {
    const int w = __atomic_load_n(&mh->seq, __ATOMIC_ACQUIRE);
    *slot = w >> 2;
    *state = w & 3;
}

namespace {

constexpr int kGmThreads = 512;
// dynamic LDS of the iteration kernel: the new vector and staged basis vectors
constexpr size_t kGmIterLds = 131072;
// dynamic LDS of the slot control kernel: the working vector and the staged
// basis (its static LDS, under 16 KB, fills the CU's 160 KB)
constexpr size_t kGmSlotLds = 147456;


// sixteen wavefront sums at once by a butterfly that halves the values per
// lane at each exchange (8 + 4 + 2 + 1 + 2 exchanges instead of 16 x 6):
// lane l returns the total of v[(l >> 2) & 15]
template <class T>
__device__ inline T wave_sum16(T (&v)[16], int lane) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const bool hi = lane & 32;
        const T send = hi ? v[i] : v[i + 8];
        const T keep = hi ? v[i + 8] : v[i];
        v[i] = keep + xl<5>(send);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const bool hi = lane & 16;
        const T send = hi ? v[i] : v[i + 4];
        const T keep = hi ? v[i + 4] : v[i];
        v[i] = keep + xl<4>(send);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const bool hi = lane & 8;
        const T send = hi ? v[i] : v[i + 2];
        const T keep = hi ? v[i + 2] : v[i];
        v[i] = keep + xl<3>(send);
    }
    {
        const bool hi = lane & 4;
        const T send = hi ? v[0] : v[1];
        const T keep = hi ? v[1] : v[0];
        v[0] = keep + xl<2>(send);
    }
    v[0] += xl<1>(v[0]);
    v[0] += xl<0>(v[0]);
    return v[0];
}

// K wavefront sums at once (K = 4, 8): the butterfly of wave_sum16 with
// log2 K halving exchanges, then full exchanges over the remaining lane bits;
// lane l returns the total of v[(l >> (6 - log2 K)) & (K - 1)]
template <int B, int H, class T, int K>
__device__ __forceinline__ void halve_at(T (&v)[K], int lane) {
    const bool hi = (lane >> B) & 1;
#pragma unroll
    for (int i = 0; i < H; ++i) {
        const T send = hi ? v[i] : v[i + H];
        const T keep = hi ? v[i + H] : v[i];
        v[i] = keep + xl<B>(send);
    }
}
template <int K, class T>
__device__ inline T wave_sum_k(T (&v)[K], int lane) {
    if constexpr (K == 16) {
        return wave_sum16(v, lane);
    } else if constexpr (K == 8) {
        halve_at<5, 4>(v, lane);
        halve_at<4, 2>(v, lane);
        halve_at<3, 1>(v, lane);
        v[0] += xl<2>(v[0]);
        v[0] += xl<1>(v[0]);
        v[0] += xl<0>(v[0]);
        return v[0];
    } else {
        static_assert(K == 4, "K = 4, 8 or 16");
        halve_at<5, 2>(v, lane);
        halve_at<4, 1>(v, lane);
        v[0] += xl<3>(v[0]);
        v[0] += xl<2>(v[0]);
        v[0] += xl<1>(v[0]);
        v[0] += xl<0>(v[0]);
        return v[0];
    }
}

// block-wide sum; every thread gets the result
template <class T>
__device__ T block_sum(T v, T *red) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    v = wave_sum(v);
    if (lane == 0) red[wid] = v;
    __syncthreads();
    T s = zero<T>();
    const int nw = blockDim.x >> 6;
    for (int q = 0; q < nw; ++q) s += red[q];
    __syncthreads();
    return s;
}

__device__ inline double absv(double a) { return fabs(a); }
__device__ inline double absv(cd a) { return hypot(a.x, a.y); }
__device__ inline double re_part(double a) { return a; }
__device__ inline double re_part(cd a) { return a.x; }

template <class T> __device__ inline T scale_of(double s);
template <> __device__ inline double scale_of<double>(double s) { return s; }
template <> __device__ inline cd scale_of<cd>(double s) { return make_cd(s, 0.0); }

// ||b|| into the control block
template <class T>
__global__ __launch_bounds__(kGmThreads) void k_gm_bnorm(GmCtl *ctl, const T *b, int Nb) {
    __shared__ double red[16];
    double s = 0.0;
    for (int i = threadIdx.x; i < Nb; i += blockDim.x) s += abs2(b[i]);
    s = block_sum(s, red);
    if (threadIdx.x == 0) ctl->bnorm = sqrt(s);
}

// start of a cycle: v_0 = r/||r||, g = ||r|| e_1
template <class T>
__global__ __launch_bounds__(kGmThreads) void k_gm_start(GmCtl *ctl, const T *r, T *V, T *g, int Nb) {
    __shared__ double red[16];
    double s = 0.0;
    for (int i = threadIdx.x; i < Nb; i += blockDim.x) s += abs2(r[i]);
    s = block_sum(s, red);
    const double beta = sqrt(s);
    const int limit = ctl->fixed > 0 ? ctl->fixed : ctl->max_iter;
    const bool conv = beta <= ctl->tol * ctl->bnorm;
    const bool stop = (ctl->fixed == 0 && conv) || beta == 0.0 || ctl->iters >= limit;
    if (!stop) {
        const double inv = 1.0 / beta;
        for (int i = threadIdx.x; i < Nb; i += blockDim.x) V[i] = r[i] * inv;
    }
    if (threadIdx.x == 0) {
        for (int q = 0; q <= ctl->m; ++q) g[q] = zero<T>();
        g[0] = scale_of<T>(beta);
        ctl->beta = beta;
        ctl->resid = beta;
        ctl->j = 0;
        ctl->breakdown = 0;
        ctl->converged = conv ? 1 : 0;
        ctl->done = stop ? 1 : 0;
    }
}

// one Arnoldi step on column j: w = V[j+1] holds K v_j on entry
template <class T, int EPT>
__global__ __launch_bounds__(kGmThreads) void k_gm_arnoldi(GmCtl *ctl, T *V, T *H, T *g, double *cs, T *sn,
                                                           int Nb) {
    if (ctl->done) return;
    __shared__ T red[16][8];
    __shared__ T hs[72];
    __shared__ double redd[16];
    const int j = ctl->j, m = ctl->m;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    T *w = V + (size_t)(j + 1) * Nb;
    T wl[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        int idx = tid + e * kGmThreads;
        wl[e] = idx < Nb ? w[idx] : zero<T>();
    }
    for (int pass = 0; pass < 2; ++pass) {
        for (int i0 = 0; i0 <= j; i0 += 8) {
            T part[8];
#pragma unroll
            for (int ii = 0; ii < 8; ++ii) part[ii] = zero<T>();
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                int idx = tid + e * kGmThreads;
                if (idx < Nb) {
#pragma unroll
                    for (int ii = 0; ii < 8; ++ii)
                        if (i0 + ii <= j) part[ii] += conjv(V[(size_t)(i0 + ii) * Nb + idx]) * wl[e];
                }
            }
#pragma unroll
            for (int ii = 0; ii < 8; ++ii) {
                T s = wave_sum(part[ii]);
                if (lane == 0) red[wid][ii] = s;
            }
            __syncthreads();
            if (tid < 8 && i0 + tid <= j) {
                T s = zero<T>();
                for (int q = 0; q < (kGmThreads >> 6); ++q) s += red[q][tid];
                hs[i0 + tid] = s;
                size_t hidx = (size_t)(i0 + tid) * m + j;
                H[hidx] = pass == 0 ? s : H[hidx] + s;
            }
            __syncthreads();
        }
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            int idx = tid + e * kGmThreads;
            if (idx < Nb)
                for (int i = 0; i <= j; ++i) wl[e] -= hs[i] * V[(size_t)i * Nb + idx];
        }
        __syncthreads();
    }
    double s2 = 0.0;
#pragma unroll
    for (int e = 0; e < EPT; ++e) s2 += abs2(wl[e]);
    const double hn = sqrt(block_sum(s2, redd));
    if (hn > 0.0) {
        const double inv = 1.0 / hn;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            int idx = tid + e * kGmThreads;
            if (idx < Nb) w[idx] = wl[e] * inv;
        }
    }
    __syncthreads();
    if (tid == 0) {
        H[(size_t)(j + 1) * m + j] = scale_of<T>(hn);
        for (int i = 0; i < j; ++i) {
            T a = H[(size_t)i * m + j], b = H[(size_t)(i + 1) * m + j];
            H[(size_t)i * m + j] = a * cs[i] + sn[i] * b;
            H[(size_t)(i + 1) * m + j] = b * cs[i] - conjv(sn[i]) * a;
        }
        T a = H[(size_t)j * m + j];
        const double bb = hn;
        const double aa = absv(a);
        const double rho = hypot(aa, bb);
        double c;
        T s;
        if (aa == 0.0) {
            c = 0.0;
            s = scale_of<T>(1.0);
        } else {
            c = aa / rho;
            s = a * (bb / (aa * rho));   // (a/|a|) conj(b)/rho with b real
        }
        cs[j] = c;
        sn[j] = s;
        H[(size_t)j * m + j] = a * c + s * bb;
        H[(size_t)(j + 1) * m + j] = zero<T>();
        T gj = g[j];
        g[j + 1] = -(conjv(s) * gj);
        g[j] = gj * c;
        const double resid = absv(g[j + 1]);
        ctl->resid = resid;
        const int it = ctl->iters + 1;
        ctl->iters = it;
        ctl->j = j + 1;
        const bool conv = resid <= ctl->tol * ctl->bnorm;
        ctl->converged = conv ? 1 : 0;
        const int limit = ctl->fixed > 0 ? ctl->fixed : ctl->max_iter;
        if (hn == 0.0) ctl->breakdown = 1;
        if ((ctl->fixed == 0 && conv) || it >= limit || j + 1 >= m || hn == 0.0) ctl->done = 1;
    }
}

// ---------------------------------------------------------------------------
// Fast path with the merged corrections operator: one 16-point window of phi
// per irregular node, phi read from LDS.
// ---------------------------------------------------------------------------
constexpr int kWin = 16;

// U nodes per thread per round: all their coefficient loads are issued
// before the first use, so a round costs one memory latency
template <class T>
__device__ void corr_merged_block(const T *phi_lds, int Nb, int n_irr, const T *__restrict__ mcoef,
                                  const int32_t *__restrict__ mbase, T *__restrict__ corr, int q_first = 0) {
    constexpr int U = sizeof(T) == 8 ? 4 : 2;
    const int nt = blockDim.x;
    for (int q0 = q_first + threadIdx.x; q0 < n_irr; q0 += U * nt) {
        T c[U][kWin];
        int b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int q = q0 + u * nt;
            b[u] = 0;
            if (q < n_irr) {
                b[u] = mbase[q];
#pragma unroll
                for (int o = 0; o < kWin; ++o) c[u][o] = mcoef[(size_t)o * n_irr + q];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int q = q0 + u * nt;
            if (q < n_irr) {
                T acc = zero<T>();
#pragma unroll
                for (int o = 0; o < kWin; ++o) {
                    int idx = b[u] + o;
                    if (idx >= Nb) idx -= Nb;
                    acc += c[u][o] * phi_lds[idx];
                }
                corr[q] = acc;
            }
        }
    }
}

// corrections of an explicit density (the current iterate), many workgroups
template <class T>
__global__ void k_corr_merged(const T *__restrict__ phi, int Nb, int n_irr, const T *__restrict__ mcoef,
                              const int32_t *__restrict__ mbase, T *__restrict__ corr) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_irr) return;
    const int b = mbase[q];
    T acc = zero<T>();
#pragma unroll
    for (int o = 0; o < kWin; ++o) {
        int idx = b + o;
        if (idx >= Nb) idx -= Nb;
        acc += mcoef[(size_t)o * n_irr + q] * phi[idx];
    }
    corr[q] = acc;
}

// extraction K phi at collocation point k from the grid values at its stencil
template <class T>
__device__ inline T extract_k(int k, int Nb, const T *__restrict__ ust, const double *__restrict__ w6,
                              const T *__restrict__ bop, const T *__restrict__ phi) {
    T acc = zero<T>();
#pragma unroll
    for (int p = 0; p < 6; ++p) acc = mad_(ust[6 * k + p], w6[6 * k + p], acc);
#pragma unroll
    for (int o = 0; o < 5; ++o) {
        int idx = k - 2 + o;
        idx = idx < 0 ? idx + Nb : (idx >= Nb ? idx - Nb : idx);
        acc = mad_(bop[5 * k + o], phi[idx], acc);
    }
    return acc;
}

// Start of a cycle: r = b - K x (extraction of the product whose grid solve
// has just run), beta = ||r||, v_0 = r / beta, g = beta e_1, and the
// corrections of v_0 for the first product of the cycle.  Dynamic LDS:
// Nb elements.
template <class T>
__global__ __launch_bounds__(kGmThreads) void k_gm_start_res(GmCtl *ctl, const T *__restrict__ x,
                                                             const T *__restrict__ b, T *V, T *g, int Nb,
                                                             const T *__restrict__ ust, const double *__restrict__ w6,
                                                             const T *__restrict__ bop, int n_irr,
                                                             const T *__restrict__ mcoef,
                                                             const int32_t *__restrict__ mbase, T *corr) {
    extern __shared__ double dyn[];
    T *sv = reinterpret_cast<T *>(dyn);
    __shared__ double red[16];
    __shared__ int sstop;
    double s = 0.0;
    for (int k = threadIdx.x; k < Nb; k += blockDim.x) {
        const T r = b[k] - extract_k(k, Nb, ust, w6, bop, x);
        sv[k] = r;
        s += abs2(r);
    }
    s = block_sum(s, red);
    const double beta = sqrt(s);
    const int limit = ctl->fixed > 0 ? ctl->fixed : ctl->max_iter;
    const bool conv = beta <= ctl->tol * ctl->bnorm;
    const bool stop = (ctl->fixed == 0 && conv) || beta == 0.0 || ctl->iters >= limit;
    const double inv = stop ? 0.0 : 1.0 / beta;
    for (int k = threadIdx.x; k < Nb; k += blockDim.x) {
        const T v = sv[k] * inv;
        sv[k] = v;
        V[k] = v;
    }
    if ((int)threadIdx.x <= ctl->m) g[threadIdx.x] = threadIdx.x == 0 ? scale_of<T>(beta) : zero<T>();
    if (threadIdx.x == 0) {
        ctl->beta = beta;
        ctl->resid = beta;
        ctl->j = 0;
        ctl->breakdown = 0;
        ctl->converged = conv ? 1 : 0;
        ctl->done = stop ? 1 : 0;
        const double t0 = ctl->tol * ctl->bnorm, t1 = ctl->eta * beta;
        ctl->thresh = t1 > t0 ? t1 : t0;
        sstop = stop ? 1 : 0;
    }
    __syncthreads();
    if (!sstop) corr_merged_block(sv, Nb, n_irr, mcoef, mbase, corr);
}

// One GMRES iteration after the grid solve of v_j (j is the launch's position
// in the cycle, passed by the host; launches after the cycle has finished
// find the done flag set and return):
//   extraction of w = K v_j, CGS2 against v_0..v_j, normalisation, Givens
//   update of column j and of the residual estimate, and the corrections of
//   v_{j+1} for the next product.
// All loads that do not depend on the done flag are issued before it is
// tested: the extracted vector and the first nvl basis vectors go to LDS
// (dynamic LDS: (1 + nvl) * Nb elements), so each Gram-Schmidt sweep is one
// pass of dot products, one block reduction for all of them and one update.
template <class T, int EPT>
__global__ __launch_bounds__(kGmThreads) void k_gm_iter(GmCtl *ctl, T *V, T *H, T *g, double *cs, T *sn, int Nb,
                                                        int j_arg, int m, int nvl, const T *__restrict__ ust,
                                                        const double *__restrict__ w6, const T *__restrict__ bop,
                                                        int n_irr, const T *__restrict__ mcoef,
                                                        const int32_t *__restrict__ mbase, T *corr) {
    extern __shared__ double dyn[];
    T *sw = reinterpret_cast<T *>(dyn);  // Nb: the new basis vector
    T *sV = sw + Nb;                     // nvl * Nb: v_0 .. v_{nvl-1}
    __shared__ T red[kGmThreads / 64][65];
    __shared__ T hcol[72];
    __shared__ T hs[72];
    __shared__ T ssn[72];
    __shared__ double scs[72];
    __shared__ double redd[16];
    __shared__ T sg;
    __shared__ int sdone;
    const int j = j_arg < m - 1 ? j_arg : m - 1;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int done_flag = ctl->done;
    const T *vj = V + (size_t)j * Nb;
    T *w = V + (size_t)(j + 1) * Nb;
    if (tid < j) {
        scs[tid] = cs[tid];
        ssn[tid] = sn[tid];
    }
    if (tid == 0) sg = g[j];
    const int nst = j + 1 < nvl ? j + 1 : nvl;
    for (int q = tid; q < nst * Nb; q += kGmThreads) sV[q] = V[q];
    // the first irregular node's correction window of this thread
    T cpre[kWin];
    int bpre = 0;
    if (tid < n_irr) {
        bpre = mbase[tid];
#pragma unroll
        for (int o = 0; o < kWin; ++o) cpre[o] = mcoef[(size_t)o * n_irr + tid];
    }
    for (int k = tid; k < Nb; k += kGmThreads) sw[k] = extract_k(k, Nb, ust, w6, bop, vj);
    if (done_flag) return;
    __syncthreads();
    T wl[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int k = tid + e * kGmThreads;
        wl[e] = k < Nb ? sw[k] : zero<T>();
    }
    // CGS2: h = V^H w, w -= V h, twice
    for (int pass = 0; pass < 2; ++pass) {
        for (int i0 = 0; i0 <= j; i0 += 16) {
            T part[16];
#pragma unroll
            for (int ii = 0; ii < 16; ++ii) part[ii] = zero<T>();
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const int idx = tid + e * kGmThreads;
                if (idx < Nb) {
#pragma unroll
                    for (int ii = 0; ii < 16; ++ii)
                        if (i0 + ii < nst) part[ii] += conjv(sV[(size_t)(i0 + ii) * Nb + idx]) * wl[e];
#pragma unroll
                    for (int ii = 0; ii < 16; ++ii)
                        if (i0 + ii >= nst && i0 + ii <= j)
                            part[ii] += conjv(V[(size_t)(i0 + ii) * Nb + idx]) * wl[e];
                }
            }
            const T sum = wave_sum16(part, lane);
            const int ii = (lane >> 2) & 15;
            if ((lane & 3) == 0 && i0 + ii <= j) red[wid][i0 + ii] = sum;
        }
        __syncthreads();
        if (tid <= j) {
            T sum = zero<T>();
            for (int q = 0; q < (kGmThreads >> 6); ++q) sum += red[q][tid];
            hs[tid] = sum;
            hcol[tid] = pass == 0 ? sum : hcol[tid] + sum;
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int idx = tid + e * kGmThreads;
            if (idx < Nb) {
                for (int i = 0; i < nst; ++i) wl[e] -= hs[i] * sV[(size_t)i * Nb + idx];
                for (int i = nst; i <= j; ++i) wl[e] -= hs[i] * V[(size_t)i * Nb + idx];
            }
        }
    }
    double s2 = 0.0;
#pragma unroll
    for (int e = 0; e < EPT; ++e) s2 += abs2(wl[e]);
    const double hn = sqrt(block_sum(s2, redd));
    const double inv = hn > 0.0 ? 1.0 / hn : 0.0;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int idx = tid + e * kGmThreads;
        if (idx < Nb) {
            const T v = wl[e] * inv;
            w[idx] = v;
            sw[idx] = v;
        }
    }
    if (tid == 0) {
        for (int i = 0; i < j; ++i) {
            const T a = hcol[i], b = hcol[i + 1];
            hcol[i] = a * scs[i] + ssn[i] * b;
            hcol[i + 1] = b * scs[i] - conjv(ssn[i]) * a;
        }
        const T a = hcol[j];
        const double bb = hn;
        const double aa = absv(a);
        const double rho = hypot(aa, bb);
        double c;
        T s;
        if (aa == 0.0) {
            c = 0.0;
            s = scale_of<T>(1.0);
        } else {
            c = aa / rho;
            s = a * (bb / (aa * rho));
        }
        cs[j] = c;
        sn[j] = s;
        hcol[j] = a * c + s * bb;
        hcol[j + 1] = zero<T>();
        const T gj = sg;
        const T gj1 = -(conjv(s) * gj);
        g[j + 1] = gj1;
        g[j] = gj * c;
        const double resid = absv(gj1);
        ctl->resid = resid;
        const int it = ctl->iters + 1;
        ctl->iters = it;
        ctl->j = j + 1;
        const bool conv = resid <= ctl->thresh;
        ctl->converged = (conv && ctl->eta == 0.0) ? 1 : 0;
        const int limit = ctl->fixed > 0 ? ctl->fixed : ctl->max_iter;
        if (hn == 0.0) ctl->breakdown = 1;
        const bool dn = (ctl->fixed == 0 && conv) || it >= limit || j + 1 >= m || hn == 0.0;
        ctl->done = dn ? 1 : 0;
        sdone = dn ? 1 : 0;
    }
    __syncthreads();
    if (tid <= j + 1) H[(size_t)tid * m + j] = hcol[tid];
    if (!sdone) {
        if (tid < n_irr) {
            T acc = zero<T>();
#pragma unroll
            for (int o = 0; o < kWin; ++o) {
                int idx = bpre + o;
                if (idx >= Nb) idx -= Nb;
                acc += cpre[o] * sw[idx];
            }
            corr[tid] = acc;
        }
        corr_merged_block(sw, Nb, n_irr, mcoef, mbase, corr, kGmThreads);
    }
}

// end of a cycle: y = H^{-1} g on the leading j x j block, x += V y (and,
// on the fast path, the corrections of the updated x for the next residual)
template <class T>
__global__ __launch_bounds__(kGmThreads) void k_gm_update(GmCtl *ctl, const T *V, const T *H, const T *g, T *y,
                                                          T *x, int Nb, int n_irr, const T *mcoef, const int32_t *mbase,
                                                          T *corr) {
    __shared__ T ys[72];
    __shared__ T hrow[72];
    const int jj = ctl->j, m = ctl->m;
    for (int i = jj - 1; i >= 0; --i) {
        if ((int)threadIdx.x < jj) hrow[threadIdx.x] = H[(size_t)i * m + threadIdx.x];
        __syncthreads();
        if (threadIdx.x == 0) {
            T s = g[i];
            for (int l = i + 1; l < jj; ++l) s -= hrow[l] * ys[l];
            ys[i] = s / hrow[i];
            y[i] = ys[i];
        }
        __syncthreads();
    }
    for (int idx = threadIdx.x; idx < Nb; idx += blockDim.x) {
        T acc = x[idx];
        for (int i = 0; i < jj; ++i) acc += V[(size_t)i * Nb + idx] * ys[i];
        x[idx] = acc;
    }
    if (mcoef) {
        __syncthreads();
        for (int q = threadIdx.x; q < n_irr; q += blockDim.x) {
            const int b = mbase[q];
            T acc = zero<T>();
#pragma unroll
            for (int o = 0; o < kWin; ++o) {
                int idx = b + o;
                if (idx >= Nb) idx -= Nb;
                acc += mcoef[(size_t)o * n_irr + q] * x[idx];
            }
            corr[q] = acc;
        }
    }
}

// ---------------------------------------------------------------------------
// Device-driven GMRES (merged-operator path)
// ---------------------------------------------------------------------------

// gate words of the next slot for a new state
__device__ inline void gm_set_state(GmCtl *ctl, int st) {
    ctl->state = st;
    ctl->skip64 = (st == kStDone || (st == kStIter && ctl->mixed)) ? 1 : 0;
    ctl->skip32 = (st == kStIter && ctl->mixed) ? 0 : 1;
    ctl->skip_tail = st == kStDone ? 0 : 1;
}

// The mirror is fine-grained (uncached) host memory: the fields are plain
// stores, and waiting for their completion before the store of seq orders
// them for the host without a release fence (which would write back the
// whole L2 of the XCD).
__device__ inline void gm_publish(GmCtl *ctl, GmMirror *mir) {
    mir->state = ctl->state;
    mir->iters = ctl->iters;
    mir->converged = ctl->converged;
    mir->cycles = ctl->cycles;
    mir->resid = ctl->resid;
    mir->bnorm = ctl->bnorm;
    __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __hip_atomic_store(&mir->seq, 4 * ctl->slot + ctl->state, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// control block, ||b||, and x_0 as the first slot's density
template <class T>
struct GmInitArgs {
    const int *off;  // nonzero: member not solved in this call (batched solves)
    GmCtl *ctl;
    const T *b;
    T *x;
    const T *x0;  // the start: == x (already in place), another array (copied
                  // into x), or null (zero)
    T *vcur;
    int Nb, max_iter, m, fixed;
    double tol, eta;
    int mixed;
};

template <class T>
__device__ void gm_init_body(const GmInitArgs<T> &A, int) {
    if (A.off && *A.off) return;
    GmCtl *ctl = A.ctl;
    const T *__restrict__ b = A.b;
    T *x = A.x;
    const T *x0 = A.x0;
    T *__restrict__ vcur = A.vcur;
    const int Nb = A.Nb, max_iter = A.max_iter, m = A.m, fixed = A.fixed, mixed = A.mixed;
    const double tol = A.tol, eta = A.eta;
    __shared__ double red[16];
    double s = 0.0;
    for (int k = threadIdx.x; k < Nb; k += blockDim.x) {
        s += abs2(b[k]);
        T v;
        if (x0 == x) {
            v = x[k];
        } else {
            v = x0 ? x0[k] : zero<T>();
            x[k] = v;
        }
        vcur[k] = v;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) {
        ctl->j = 0;
        ctl->done = 0;
        ctl->iters = 0;
        ctl->converged = 0;
        ctl->max_iter = max_iter;
        ctl->m = m;
        ctl->fixed = fixed;
        ctl->breakdown = 0;
        ctl->tol = tol;
        ctl->bnorm = sqrt(s);
        ctl->beta = 0.0;
        ctl->resid = 0.0;
        ctl->eta = eta;
        ctl->thresh = 0.0;
        ctl->slot = 0;
        ctl->cycles = 0;
        ctl->mixed = mixed;
        ctl->pad = 0;
        gm_set_state(ctl, kStStart);
    }
}

template <class T>
__global__ __launch_bounds__(kGmThreads) void k_gm_init(GmInitArgs<T> A) {
    gm_init_body(A, 0);
}

// The control kernel of one slot (see the schedule above).  kv holds K vcur
// from the slot's grid solve; the kernel ends by writing the density of the
// next product to vcur.  Dynamic LDS: [Nb: working vector][nvl*Nb: staged
// basis][m*m: triangular factor at a cycle end].
template <class T>
struct SlotArgs {
    const int *off;  // nonzero: member not solved in this call (batched solves)
    int replay;      // nonzero: timing replay, the control block is not advanced
    int quiet;       // nonzero: publish to the host mirror only when the solve
                     // finishes (the host reads the mirror once a batch of
                     // slots has run; the batch's last slot is not quiet)
    GmCtl *ctl;
    GmMirror *mir;
    T *V, *H, *g;
    double *cs;
    T *sn, *x;
    const T *b;
    T *vcur;
    const T *kv;
    int Nb, m, nvl;
};

template <class T, int EPT>
__device__ void gm_slot_body(const SlotArgs<T> &A, int) {
    if (A.off && *A.off) return;
    GmCtl *ctl = A.ctl;
    GmMirror *mir = A.mir;
    T *V = A.V, *H = A.H, *g = A.g, *sn = A.sn, *x = A.x;
    double *cs = A.cs;
    const T *__restrict__ b = A.b;
    T *__restrict__ vcur = A.vcur;
    const T *__restrict__ kv = A.kv;
    const int Nb = A.Nb, m = A.m, nvl = A.nvl;
    extern __shared__ double dyn[];
    T *sw = reinterpret_cast<T *>(dyn);
    T *sV = sw + Nb;
    // the triangular factor of a cycle end takes the place of the staged
    // basis, which is no longer read by then
    T *sH = sV;
    __shared__ T red[kGmThreads / 64][65];
    __shared__ T hcol[72];
    __shared__ T hs[72];
    __shared__ T ssn[72];
    __shared__ T sgv[72];
    __shared__ T ys[72];
    __shared__ double scs[72];
    __shared__ double redd[16];
    __shared__ int sflag, sconv, sit;
    __shared__ double snrm;
    // one read of the control block (uniform); thread 0 writes back what
    // changes, so no control field is re-read from memory on the critical path
    const GmCtl c = *ctl;
    const int state = c.state;
    if (state == kStDone) return;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int limit = c.fixed > 0 ? c.fixed : c.max_iter;

    if (state == kStStart) {
        // r = b - K x, stop test, v_0 = r / beta, corrections of v_0
        double s = 0.0;
        for (int k = tid; k < Nb; k += kGmThreads) {
            const T r = b[k] - kv[k];
            sw[k] = r;
            s += abs2(r);
        }
        s = block_sum(s, redd);
        const double beta = sqrt(s);
        const bool conv = beta <= c.tol * c.bnorm;
        const bool stop = (c.fixed == 0 && conv) || beta == 0.0 || c.iters >= limit;
        const double inv = stop ? 0.0 : 1.0 / beta;
        for (int k = tid; k < Nb; k += kGmThreads) {
            const T v = sw[k] * inv;
            V[k] = v;
            vcur[k] = v;
        }
        if (tid <= m) g[tid] = tid == 0 ? scale_of<T>(beta) : zero<T>();
        if (tid == 0) {
            ctl->beta = beta;
            ctl->resid = beta;
            ctl->j = 0;
            ctl->breakdown = 0;
            ctl->converged = conv ? 1 : 0;
            ctl->cycles = c.cycles + 1;
            const double t0 = c.tol * c.bnorm, t1 = c.eta * beta;
            ctl->thresh = t1 > t0 ? t1 : t0;
            ctl->slot = c.slot + 1;
            gm_set_state(ctl, stop ? kStDone : kStIter);
            if (stop || !A.quiet) gm_publish(ctl, mir);
        }
        return;
    }

    // Arnoldi step on column j: w = K v_j, CGS2, Givens
    const int j = c.j;
    T *w = V + (size_t)(j + 1) * Nb;
    if (tid < j) {
        scs[tid] = cs[tid];
        ssn[tid] = sn[tid];
    }
    if (tid <= j) sgv[tid] = g[tid];
    const int nst = j + 1 < nvl ? j + 1 : nvl;
    // the thread's elements of w = K v_j straight into registers, and the
    // basis staged in LDS with sixteen loads in flight per thread (clamped,
    // in bounds) before the LDS writes: every load is issued before the
    // first wait, so the set-up costs about one memory round trip
    T wl[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int k = tid + e * kGmThreads;
        const T x = kv[min(k, Nb - 1)];
        wl[e] = k < Nb ? x : zero<T>();
    }
    {
        const int total = nst * Nb;
        for (int q0 = tid; q0 < total; q0 += 16 * kGmThreads) {
            T v16[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) v16[u] = V[min(q0 + u * kGmThreads, total - 1)];
#pragma unroll
            for (int u = 0; u < 16; ++u)
                if (q0 + u * kGmThreads < total) sV[q0 + u * kGmThreads] = v16[u];
        }
    }
    __syncthreads();
    // CGS2 against v_0..v_j.  All of v_0..v_j staged: branch-free dot
    // products (clamped LDS reads, masked terms) so that every read is in
    // flight before the first use.
    const bool staged = j + 1 <= nst;
    for (int pass = 0; pass < 2; ++pass) {
        // each pass also forms the squared norm of its input (slot j + 1 of
        // its reduction): the first decides whether a second pass is needed,
        // the last gives the norm of the result without a reduction of its
        // own
        const int jn = j + 1;
        // the products in chunks of 4, 8 or 16 (the fewest that cover the
        // jn + 1 terms, so that few lanes of the reduction carry zeros)
        auto chunk = [&](auto kk, int i0) {
            constexpr int K = decltype(kk)::value;
            T part[K];
#pragma unroll
            for (int ii = 0; ii < K; ++ii) part[ii] = zero<T>();
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const int idx = tid + e * kGmThreads;
                if (idx < Nb) {
                    T vv[K];
#pragma unroll
                    for (int ii = 0; ii < K; ++ii) {
                        const int i = i0 + ii <= j ? i0 + ii : j;
                        vv[ii] = sV[(size_t)i * Nb + idx];
                    }
#pragma unroll
                    for (int ii = 0; ii < K; ++ii)
                        part[ii] += (i0 + ii <= j ? conjv(vv[ii]) : (i0 + ii == jn ? conjv(wl[e]) : zero<T>())) *
                                    wl[e];
                }
            }
            const T sum = wave_sum_k<K>(part, lane);
            constexpr int S = K == 16 ? 2 : (K == 8 ? 3 : 4);
            const int ii = (lane >> S) & (K - 1);
            if ((lane & ((1 << S) - 1)) == 0 && i0 + ii <= jn) red[wid][i0 + ii] = sum;
        };
        for (int i0 = 0; i0 <= jn && staged;) {
            const int rem = jn + 1 - i0;
            if (rem <= 4) {
                chunk(std::integral_constant<int, 4>(), i0);
                i0 += 4;
            } else if (rem <= 8) {
                chunk(std::integral_constant<int, 8>(), i0);
                i0 += 8;
            } else {
                chunk(std::integral_constant<int, 16>(), i0);
                i0 += 16;
            }
        }
        for (int i0 = 0; i0 <= jn && !staged; i0 += 16) {
            T part[16];
#pragma unroll
            for (int ii = 0; ii < 16; ++ii) part[ii] = zero<T>();
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const int idx = tid + e * kGmThreads;
                if (idx < Nb) {
#pragma unroll
                    for (int ii = 0; ii < 16; ++ii)
                        if (i0 + ii < nst) part[ii] += conjv(sV[(size_t)(i0 + ii) * Nb + idx]) * wl[e];
#pragma unroll
                    for (int ii = 0; ii < 16; ++ii)
                        if (i0 + ii >= nst && i0 + ii <= j)
                            part[ii] += conjv(V[(size_t)(i0 + ii) * Nb + idx]) * wl[e];
#pragma unroll
                    for (int ii = 0; ii < 16; ++ii)
                        if (i0 + ii > j && i0 + ii == jn) part[ii] += conjv(wl[e]) * wl[e];
                }
            }
            const T sum = wave_sum16(part, lane);
            const int ii = (lane >> 2) & 15;
            if ((lane & 3) == 0 && i0 + ii <= jn) red[wid][i0 + ii] = sum;
        }
        __syncthreads();
        if (tid <= j) {
            T sum = zero<T>();
            for (int q = 0; q < (kGmThreads >> 6); ++q) sum += red[q][tid];
            hs[tid] = sum;
            hcol[tid] = pass == 0 ? sum : hcol[tid] + sum;
        } else if (tid == jn) {
            T sum = zero<T>();
            for (int q = 0; q < (kGmThreads >> 6); ++q) sum += red[q][tid];
            snrm = re_part(sum);
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int idx = tid + e * kGmThreads;
            if (idx < Nb) {
                if (staged) {
                    for (int i0 = 0; i0 <= j; i0 += 4) {
                        T vv[4], hh[4];
#pragma unroll
                        for (int ii = 0; ii < 4; ++ii) {
                            const int i = i0 + ii <= j ? i0 + ii : j;
                            vv[ii] = sV[(size_t)i * Nb + idx];
                            hh[ii] = i0 + ii <= j ? hs[i] : zero<T>();
                        }
#pragma unroll
                        for (int ii = 0; ii < 4; ++ii) wl[e] -= hh[ii] * vv[ii];
                    }
                } else {
                    for (int i = 0; i < nst; ++i) wl[e] -= hs[i] * sV[(size_t)i * Nb + idx];
                    for (int i = nst; i <= j; ++i) wl[e] -= hs[i] * V[(size_t)i * Nb + idx];
                }
            }
        }
        // the second pass (Daniel, Gragg, Kaufman and Stewart's criterion)
        // only when the first removed more than half of ||w||^2, i.e. when
        // ||w'|| = sqrt(||w||^2 - sum |h_i|^2) <= ||w|| / sqrt(2): otherwise
        // w' is orthogonal to the basis to working precision already.  The
        // values are in LDS, so every thread takes the same branch.
        if (pass == 0) {
            double r2 = snrm;
            for (int i = 0; i <= j; ++i) r2 -= abs2(hs[i]);
            if (r2 > 0.5 * snrm) break;
        }
    }
    // The result's norm from the last pass: ||out||^2 = ||in||^2 - sum |h_i|^2
    // (out = in - sum h_i v_i, the v_i orthonormal), unless that pass
    // removed half of ||in||^2 or more (only possible after a second pass
    // when w' lay almost in the span); then it is summed directly.  Every
    // thread forms the same value from LDS, so the branch is uniform.
    double hn2 = snrm;
    for (int i = 0; i <= j; ++i) hn2 -= abs2(hs[i]);
    double hn;
    if (hn2 > 0.5 * snrm) {
        hn = sqrt(hn2);
    } else {
        double s2 = 0.0;
#pragma unroll
        for (int e = 0; e < EPT; ++e) s2 += abs2(wl[e]);
        hn = sqrt(block_sum(s2, redd));
    }
    const double inv = hn > 0.0 ? 1.0 / hn : 0.0;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int idx = tid + e * kGmThreads;
        if (idx < Nb) {
            const T v = wl[e] * inv;
            w[idx] = v;
            vcur[idx] = v;
        }
    }
    if (tid == 0) {
        for (int i = 0; i < j; ++i) {
            const T a = hcol[i], bb = hcol[i + 1];
            hcol[i] = a * scs[i] + ssn[i] * bb;
            hcol[i + 1] = bb * scs[i] - conjv(ssn[i]) * a;
        }
        const T a = hcol[j];
        const double aa = absv(a);
        const double rho = hypot(aa, hn);
        double cg;
        T sr;
        if (aa == 0.0) {
            cg = 0.0;
            sr = scale_of<T>(1.0);
        } else {
            cg = aa / rho;
            sr = a * (hn / (aa * rho));
        }
        cs[j] = cg;
        sn[j] = sr;
        hcol[j] = a * cg + sr * hn;
        hcol[j + 1] = zero<T>();
        const T gj = sgv[j];
        const T gj1 = -(conjv(sr) * gj);
        g[j + 1] = gj1;
        g[j] = gj * cg;
        sgv[j] = gj * cg;
        const double resid = absv(gj1);
        const int it = c.iters + 1;
        const bool conv = resid <= c.thresh;
        const int converged = (conv && c.eta == 0.0) ? 1 : 0;
        if (!A.replay) {
            ctl->resid = resid;
            ctl->iters = it;
            ctl->j = j + 1;
            ctl->converged = converged;
            if (hn == 0.0) ctl->breakdown = 1;
        }
        const bool end = (c.fixed == 0 && conv) || it >= limit || j + 1 >= m || hn == 0.0;
        sflag = end ? 1 : 0;
        sconv = converged;
        sit = it;
    }
    __syncthreads();
    if (tid <= j + 1) H[(size_t)tid * m + j] = hcol[tid];
    if (!sflag) {
        // next Arnoldi step on v_{j+1} (already in vcur)
        if (tid == 0 && !A.replay) {
            ctl->slot = c.slot + 1;
            gm_set_state(ctl, kStIter);
            if (!A.quiet) gm_publish(ctl, mir);
        }
        return;
    }
    // end of the cycle: y = R^{-1} g on the leading (j+1) block (R is the
    // rotated Hessenberg matrix: columns 0..j-1 from earlier steps, column j
    // in hcol), x += V y, corrections of x
    const int n1 = j + 1;
    for (int q = tid; q < n1 * n1; q += kGmThreads) {
        const int r = q / n1, c = q - r * n1;
        sH[q] = c == j ? hcol[r] : H[(size_t)r * m + c];
    }
    __syncthreads();
    for (int l = j; l >= 0; --l) {
        if (tid == 0) ys[l] = sgv[l] / sH[l * n1 + l];
        __syncthreads();
        if (tid < l) sgv[tid] -= sH[tid * n1 + l] * ys[l];
        __syncthreads();
    }
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int idx = tid + e * kGmThreads;
        if (idx < Nb) {
            T acc = x[idx];
            for (int i = 0; i <= j; ++i) acc += V[(size_t)i * Nb + idx] * ys[i];
            x[idx] = acc;
            vcur[idx] = acc;
        }
    }
    if (tid == 0) {
        // FP64: the residual estimate decides; mixed: the FP64 residual of
        // the next cycle start decides
        const bool finished = sconv || sit >= limit;
        ctl->slot = c.slot + 1;
        gm_set_state(ctl, finished ? kStDone : kStStart);
        if (finished || !A.quiet) gm_publish(ctl, mir);
    }
}

template <class T, int EPT>
__global__ __launch_bounds__(kGmThreads) void k_gm_slot(SlotArgs<T> A) {
    gm_slot_body<T, EPT>(A, 0);
}

// The control kernel of one Richardson slot (eq. 3.21 as x + gamma (b - K x)).
// kv holds K x from the slot's grid solve, x the current density (equal to
// vcur).  The residual of x decides the stop; otherwise x and vcur advance.
template <class T>
struct RichArgs {
    GmCtl *ctl;
    GmMirror *mir;
    T *x, *vcur;
    const T *b, *kv;
    int Nb;
    double gamma;
};

template <class T>
__global__ __launch_bounds__(kGmThreads) void k_rich_slot(RichArgs<T> A) {
    GmCtl *ctl = A.ctl;
    const GmCtl c = *ctl;
    if (c.state == kStDone) return;
    __shared__ double red[16];
    const int Nb = A.Nb;
    double s = 0.0;
    for (int k = threadIdx.x; k < Nb; k += blockDim.x) s += abs2(A.b[k] - A.kv[k]);
    const double resid = sqrt(block_sum(s, red));
    const bool conv = resid <= c.tol * c.bnorm;
    const bool stop = c.fixed > 0 ? c.iters >= c.fixed : (conv || c.iters >= c.max_iter);
    if (!stop) {
        for (int k = threadIdx.x; k < Nb; k += blockDim.x) {
            const T xn = A.x[k] + (A.b[k] - A.kv[k]) * A.gamma;
            A.x[k] = xn;
            A.vcur[k] = xn;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        ctl->iters = c.iters + (stop ? 0 : 1);
        ctl->resid = resid;
        ctl->converged = conv ? 1 : 0;
        ctl->slot = c.slot + 1;
        gm_set_state(ctl, stop ? kStDone : kStIter);
        gm_publish(ctl, A.mir);
    }
}

struct GmPtrs {
    GmCtl *ctl;
    void *V, *H, *g, *sn, *y, *x, *b, *r;
    void *vcur;  // the density whose product the next slot computes
    double *cs;
};

GmPtrs gm_layout(kfbi_domain *d, int mmax) {
    GmPtrs P;
    const size_t es = elem_size(d), Nb = d->Nb;
    char *base = (char *)d->gm;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base + off;
        off += (bytes + 255) & ~(size_t)255;
        return (void *)p;
    };
    P.ctl = (GmCtl *)take(sizeof(GmCtl));
    P.V = take((mmax + 1) * Nb * es);
    P.H = take((size_t)(mmax + 1) * mmax * es);
    P.g = take((mmax + 1) * es);
    P.cs = (double *)take(mmax * sizeof(double));
    P.sn = take(mmax * es);
    P.y = take(mmax * es);
    P.x = take(Nb * es);
    P.b = take(Nb * es);
    P.r = take(Nb * es);
    P.vcur = take(Nb * es);
    return P;
}

}  // namespace

// the density of the last solve on this domain (Nb values, device)
const void *gmres_last_density(kfbi_domain *d) {
    if (!d->gm) return nullptr;
    GmPtrs P = gm_layout(d, 64);
    return P.x;
}

size_t gmres_bytes(kfbi_domain *d) {
    const size_t es = elem_size(d), Nb = d->Nb, mmax = 64;
    size_t tot = 0;
    auto add = [&](size_t b) { tot += (b + 255) & ~(size_t)255; };
    add(sizeof(GmCtl));
    add((mmax + 1) * Nb * es);
    add((mmax + 1) * mmax * es);
    add((mmax + 1) * es);
    add(mmax * sizeof(double));
    add(mmax * es);
    add(mmax * es);
    add(Nb * es);
    add(Nb * es);
    add(Nb * es);
    add(Nb * es);
    return tot;
}

// elements of a basis vector per thread: the smallest power of two that covers Nb
template <class T>
static int launch_arnoldi(kfbi_domain *d, GmPtrs &P, int Nb, hipStream_t s) {
    const int ept = (Nb + kGmThreads - 1) / kGmThreads;
    const int ps = prof_begin(d);
#define KFBI_ARN(E) k_gm_arnoldi<T, E><<<1, kGmThreads, 0, s>>>(P.ctl, (T *)P.V, (T *)P.H, (T *)P.g, P.cs, (T *)P.sn, Nb)
    if (ept <= 1) KFBI_ARN(1);
    else if (ept <= 2) KFBI_ARN(2);
    else if (ept <= 4) KFBI_ARN(4);
    else if (ept <= 8) KFBI_ARN(8);
    else if (ept <= 16) KFBI_ARN(16);
    else KFBI_ARN(32);
#undef KFBI_ARN
    KFBI_CHECK_LAUNCH();
    prof_end(d, ps, KFBI_K_ARNOLDI, 0.0);
    return KFBI_OK;
}

template <class T>
static int launch_iter(kfbi_domain *d, GmPtrs &P, int Nb, int j, int m, hipStream_t s) {
    const int ept = (Nb + kGmThreads - 1) / kGmThreads;
    // basis vectors staged in LDS: as many as fit beside the new vector in
    // kGmIterLds bytes
    const int jj0 = j < m - 1 ? j : m - 1;
    int nvl = (int)(kGmIterLds / ((size_t)Nb * sizeof(T))) - 1;
    if (nvl > jj0 + 1) nvl = jj0 + 1;
    if (nvl < 0) nvl = 0;
    const size_t lds = (size_t)(1 + nvl) * Nb * sizeof(T);
    const int ps = prof_begin(d);
#define KFBI_ITER(E)                                                                                            \
    k_gm_iter<T, E><<<1, kGmThreads, lds, s>>>(P.ctl, (T *)P.V, (T *)P.H, (T *)P.g, P.cs, (T *)P.sn, Nb, j, m, nvl, \
                                               (const T *)d->ust, d->w6, (const T *)d->bop, d->n_irr,            \
                                               (const T *)d->mcoef, d->mbase, (T *)d->corr)
    if (ept <= 1) KFBI_ITER(1);
    else if (ept <= 2) KFBI_ITER(2);
    else if (ept <= 4) KFBI_ITER(4);
    else if (ept <= 8) KFBI_ITER(8);
    else KFBI_ITER(16);
#undef KFBI_ITER
    KFBI_CHECK_LAUNCH();
    // algorithmic bytes: extraction inputs (six stencil values, weights and
    // the five jump coefficients per point, v_j), both Gram-Schmidt sweeps
    // over v_0..v_j, the new basis vector, the merged correction operator and
    // the corrections written
    const int jj = j < m - 1 ? j : m - 1;
    const double es = (double)sizeof(T);
    const double bytes = (double)Nb * (6.0 * es + 6.0 * 8.0 + 5.0 * es + es) + 2.0 * (jj + 1) * Nb * es +
                         (double)Nb * es + (double)d->n_irr * (kWin * es + 4.0 + es);
    prof_end(d, ps, KFBI_K_ARNOLDI, bytes);
    return KFBI_OK;
}

// K x (or b - K x when g/scale say so) for an explicit density pointer
static int matvec_explicit(kfbi_domain *d, double kre, double kim, const void *phi, const void *g,
                           double scale, void *out) {
    KFBI_TRY(compute_corrections(d, kre, kim, phi, nullptr, d->corr));
    KFBI_TRY(tridiag_solve(d, nullptr, d->corr, d->uhat));
    KFBI_TRY(eval_stencil_nodes(d, d->uhat, d->ust));
    KFBI_TRY(extract_boundary(d, kre, kim, d->ust, phi, nullptr, g, scale, out));
    return KFBI_OK;
}

template <class T>
static int gmres_run(kfbi_domain *d, double kre, double kim, GmPtrs &P, const kfbi_solve_opts &o, bool mixed,
                     int *iters_out, double *rel_out, int *conv_out, int *cycles_out) {
    hipStream_t s = d->stream;
    const int Nb = d->Nb;
    GmCtl h;
    memset(&h, 0, sizeof(h));
    h.max_iter = o.max_iter;
    h.m = o.restart;
    h.fixed = o.fixed_iters > 0 ? o.fixed_iters : 0;
    h.tol = o.tol;
    // mixed precision: each cycle reduces its FP64 residual by ~1e-5 with
    // FP32 grid solves (about the accuracy of the FP32 operator)
    h.eta = mixed ? 1e-5 : 0.0;
    KFBI_HIP(hipMemcpyAsync(P.ctl, &h, sizeof(h), hipMemcpyHostToDevice, s));
    k_gm_bnorm<T><<<1, kGmThreads, 0, s>>>(P.ctl, (const T *)P.b, Nb);
    KFBI_CHECK_LAUNCH();
    int *jptr = &P.ctl->j;
    int *done = &P.ctl->done;
    const size_t es = sizeof(T);
    const bool fast = d->op_merged && (size_t)Nb * es <= 65536;
    if (mixed && !fast) {
        set_error("mixed precision needs the merged correction operator (Nb too large or windows too wide)");
        return KFBI_ENOTSUP;
    }
    int cycles = 0;
    const int limit_all = h.fixed > 0 ? h.fixed : h.max_iter;
    if (fast) {
        k_corr_merged<T><<<(d->n_irr + 255) / 256, 256, 0, s>>>((const T *)P.x, Nb, d->n_irr,
                                                                (const T *)d->mcoef, d->mbase, (T *)d->corr);
        KFBI_CHECK_LAUNCH();
    }
    for (int cycle = 0; cycle < 100000; ++cycle) {
        // r = b - K x, then v_0 = r / ||r||
        if (fast) {
            KFBI_TRY(tridiag_solve(d, nullptr, d->corr, d->uhat));
            KFBI_TRY(eval_stencil_nodes(d, d->uhat, d->ust));
            k_gm_start_res<T><<<1, kGmThreads, Nb * es, s>>>(P.ctl, (const T *)P.x, (const T *)P.b, (T *)P.V,
                                                              (T *)P.g, Nb, (const T *)d->ust, d->w6,
                                                              (const T *)d->bop, d->n_irr, (const T *)d->mcoef,
                                                              d->mbase, (T *)d->corr);
        } else {
            KFBI_TRY(matvec_explicit(d, kre, kim, P.x, P.b, -1.0, P.r));
            k_gm_start<T><<<1, kGmThreads, 0, s>>>(P.ctl, (const T *)P.r, (T *)P.V, (T *)P.g, Nb);
        }
        KFBI_CHECK_LAUNCH();
        // enqueue the expected number of iterations (the previous solve's
        // count on this domain, or the fixed count) before the first read
        // of the control block, then smaller chunks
        int jnext = 0;
        const int cycle_start_iters = h.iters;
        int chunk = h.fixed > 0 ? h.fixed : (d->last_iters > 0 ? d->last_iters : 4);
        if (chunk > o.restart) chunk = o.restart;
        if (chunk > limit_all - h.iters) chunk = limit_all - h.iters;
        if (chunk < 1) chunk = 1;
        ++cycles;
        for (;;) {
            const int iters_before = h.iters;
            for (int c = 0; c < chunk; ++c) {
                d->prof_tag = c;
                if (fast && mixed) {
                    KFBI_TRY(tridiag_solve_low(d, d->corr, d->uhat32, done));
                    KFBI_TRY(eval_stencil_nodes_ctl(d, d->uhat32, d->ust, done, true));
                    KFBI_TRY(launch_iter<T>(d, P, Nb, jnext++, o.restart, s));
                } else if (fast) {
                    KFBI_TRY(tridiag_solve_ctl(d, nullptr, d->corr, d->uhat, done));
                    KFBI_TRY(eval_stencil_nodes_ctl(d, d->uhat, d->ust, done));
                    KFBI_TRY(launch_iter<T>(d, P, Nb, jnext++, o.restart, s));
                } else {
                    KFBI_TRY(compute_corrections_ctl(d, kre, kim, P.V, jptr, nullptr, d->corr, done));
                    KFBI_TRY(tridiag_solve_ctl(d, nullptr, d->corr, d->uhat, done));
                    KFBI_TRY(eval_stencil_nodes_ctl(d, d->uhat, d->ust, done));
                    KFBI_TRY(extract_boundary_ctl(d, kre, kim, d->ust, P.V, jptr, nullptr, nullptr, 1.0, P.V, 1,
                                                  done));
                    KFBI_TRY(launch_arnoldi<T>(d, P, Nb, s));
                }
            }
            d->prof_tag = -1;
            KFBI_HIP(hipMemcpyAsync(&h, P.ctl, sizeof(h), hipMemcpyDeviceToHost, s));
            KFBI_HIP(hipStreamSynchronize(s));
            if (d->prof_on) KFBI_TRY(prof_flush(d, h.iters - iters_before));
            if (h.done) break;
            chunk = 2;
        }
        // the first cycle's length sizes the first chunk of the next solve
        if (cycles == 1 && h.fixed == 0 && h.iters > cycle_start_iters) d->last_iters = h.iters - cycle_start_iters;
        if (h.j > 0) {
            k_gm_update<T><<<1, kGmThreads, 0, s>>>(P.ctl, (const T *)P.V, (const T *)P.H, (const T *)P.g,
                                                    (T *)P.y, (T *)P.x, Nb, d->n_irr,
                                                    fast ? (const T *)d->mcoef : nullptr, d->mbase, (T *)d->corr);
            KFBI_CHECK_LAUNCH();
        }
        const int limit = h.fixed > 0 ? h.fixed : h.max_iter;
        if ((h.fixed == 0 && h.converged) || h.iters >= limit || h.beta == 0.0 || h.j == 0) break;
    }
    *iters_out = h.iters;
    *rel_out = h.bnorm > 0 ? h.resid / h.bnorm : h.resid;
    *conv_out = h.converged;
    *cycles_out = cycles;
    return KFBI_OK;
}

// ---------------------------------------------------------------------------
// Host side of the device-driven schedule
// ---------------------------------------------------------------------------
constexpr int kTailTag = 1 << 20;

template <class T>
__global__ void k_copy_gated(int n, T *__restrict__ dst, const T *__restrict__ src, const int *done) {
    if (*done) return;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// dynamic LDS of the control kernel: the working vector, then nvl staged
// basis vectors, which the m x m triangular factor of a cycle end reuses
template <class T>
static size_t slot_lds(int Nb, int m, int *nvl_out) {
    const size_t es = sizeof(T), hb = (size_t)m * m * es, vb = (size_t)Nb * es;
    int nvl = 0;
    if (kGmSlotLds >= vb) nvl = (int)((kGmSlotLds - vb) / vb);
    if (nvl > m + 1) nvl = m + 1;
    *nvl_out = nvl;
    return vb + std::max(vb * nvl, hb);
}

template <class T>
GmInitArgs<T> gm_init_args(GmPtrs &P, int Nb, const kfbi_solve_opts &o, bool mixed, const void *x0) {
    GmInitArgs<T> A;
    A.off = nullptr;
    A.ctl = P.ctl;
    A.b = (const T *)P.b;
    A.x = (T *)P.x;
    A.x0 = (const T *)x0;
    A.vcur = (T *)P.vcur;
    A.Nb = Nb;
    A.max_iter = o.max_iter;
    A.m = o.restart;
    A.fixed = o.fixed_iters > 0 ? o.fixed_iters : 0;
    A.tol = o.tol;
    A.eta = mixed ? 1e-5 : 0.0;
    A.mixed = mixed ? 1 : 0;
    return A;
}

template <class T>
SlotArgs<T> slot_args(GmPtrs &P, GmMirror *mir, int Nb, int m, int nvl) {
    SlotArgs<T> A;
    A.off = nullptr;
    A.replay = 0;
    A.quiet = 0;
    A.ctl = P.ctl;
    A.mir = mir;
    A.V = (T *)P.V;
    A.H = (T *)P.H;
    A.g = (T *)P.g;
    A.cs = P.cs;
    A.sn = (T *)P.sn;
    A.x = (T *)P.x;
    A.b = (const T *)P.b;
    A.vcur = (T *)P.vcur;
    A.kv = (const T *)P.r;
    A.Nb = Nb;
    A.m = m;
    A.nvl = nvl;
    return A;
}

template <class T>
static bool slots_supported(kfbi_domain *d, int m) {
    int nvl;
    return d->op_merged && (size_t)d->Nb * sizeof(T) <= 65536 && slot_lds<T>(d->Nb, m, &nvl) <= kGmSlotLds;
}

template <class T>
static int launch_slot(kfbi_domain *d, GmPtrs &P, int Nb, int m, int slot_index, hipStream_t s,
                       bool replay = false, bool quiet = false) {
    int nvl;
    const size_t lds = slot_lds<T>(Nb, m, &nvl);
    const int ept = (Nb + kGmThreads - 1) / kGmThreads;
    GmMirror *mir = (GmMirror *)d->mirror_dev;
    const int ps = prof_begin(d);
    SlotArgs<T> A = slot_args<T>(P, mir, Nb, m, nvl);
    A.replay = replay ? 1 : 0;
    A.quiet = quiet ? 1 : 0;
#define KFBI_SLOT(E) k_gm_slot<T, E><<<1, kGmThreads, lds, s>>>(A)
    if (ept <= 1) KFBI_SLOT(1);
    else if (ept <= 2) KFBI_SLOT(2);
    else if (ept <= 4) KFBI_SLOT(4);
    else if (ept <= 8) KFBI_SLOT(8);
    else KFBI_SLOT(16);
#undef KFBI_SLOT
    KFBI_CHECK_LAUNCH();
    // algorithmic bytes of an Arnoldi step at j = slot_index - 1 (one cycle
    // start first): K v_j, both Gram-Schmidt sweeps over the basis, the new
    // vector (basis and vcur)
    int j = slot_index - 1;
    if (j < 0) j = 0;
    if (j > m - 1) j = m - 1;
    const double es = (double)sizeof(T);
    const double bytes = (double)Nb * es + 2.0 * (j + 1) * Nb * es + 2.0 * Nb * es;
    prof_end(d, ps, KFBI_K_ARNOLDI, bytes);
    return KFBI_OK;
}

// Enqueue slots (and after each batch the caller's final solve, gated on the
// finish flag) until the device reports the solve finished.  The host waits
// on the pinned mirror of the control block, not on the stream, so it
// returns while the final solve is still running.
template <class T, class Tail>
static int gmres_run_slots(kfbi_domain *d, GmPtrs &P, const void *x0, const kfbi_solve_opts &o, bool mixed,
                           Tail &&tail, int *iters_out, double *rel_out, int *conv_out, int *cycles_out) {
    const bool rich = (o.flags & KFBI_SOLVE_RICHARDSON) != 0;
    hipStream_t s = d->stream;
    const int Nb = d->Nb, m = o.restart;
    if (!d->mirror_host) {
        KFBI_HIP(hipHostMalloc(&d->mirror_host, sizeof(GmMirror), hipHostMallocMapped | hipHostMallocCoherent));
        memset(d->mirror_host, 0, sizeof(GmMirror));
        KFBI_HIP(hipHostGetDevicePointer(&d->mirror_dev, d->mirror_host, 0));
    }
    GmMirror *mh = (GmMirror *)d->mirror_host;
    __atomic_store_n(&mh->seq, 0, __ATOMIC_RELEASE);
    const int fixed = o.fixed_iters > 0 ? o.fixed_iters : 0;
    k_gm_init<T><<<1, kGmThreads, 0, s>>>(gm_init_args<T>(P, Nb, o, mixed, x0));
    KFBI_CHECK_LAUNCH();
    const int *skip64 = &P.ctl->skip64, *skip32 = &P.ctl->skip32, *skip_tail = &P.ctl->skip_tail;
    // first batch: the most slots any of the last four solves on this domain
    // took.  A steady count then leaves no surplus slot (each costs a gated
    // launch per kernel) and a count that varies by one is rarely short (a
    // short batch costs a wait for the host to enqueue more)
    int want = 0;
    for (int q = 0; q < 4; ++q) want = std::max(want, d->slot_hist[q]);
    if (want == 0) want = fixed > 0 ? fixed + 2 : 12;
    int n_enq = 0, last_batch = 0, seq_last = 0;
    for (int batch = 0;; ++batch) {
        last_batch = batch;
        for (int c = 0; c < want; ++c) {
            d->prof_tag = n_enq + c;
            // P.r receives K vcur
            KFBI_TRY(tridiag_solve_phi(d, P.vcur, d->uhat, skip64, false));
            KFBI_TRY(eval_extract_ctl(d, d->uhat, P.vcur, P.r, skip64, false));
            if (mixed) {
                KFBI_TRY(tridiag_solve_phi(d, P.vcur, d->uhat32, skip32, true));
                KFBI_TRY(eval_extract_ctl(d, d->uhat32, P.vcur, P.r, skip32, true));
            }
            if (rich) {
                const RichArgs<T> RA{P.ctl, (GmMirror *)d->mirror_dev, (T *)P.x, (T *)P.vcur, (const T *)P.b,
                                     (const T *)P.r, Nb, o.gamma > 0 ? o.gamma : 1.0};
                const int ps = prof_begin(d);
                k_rich_slot<T><<<1, kGmThreads, 0, s>>>(RA);
                KFBI_CHECK_LAUNCH();
                prof_end(d, ps, KFBI_K_ARNOLDI, 6.0 * Nb * sizeof(T));
            } else {
                // only the batch's last slot publishes unconditionally
                KFBI_TRY(launch_slot<T>(d, P, Nb, m, n_enq + c, s, false, c + 1 < want));
            }
        }
        n_enq += want;
        d->prof_tag = kTailTag + batch;
        KFBI_TRY(tail(skip_tail));
        d->prof_tag = -1;
        // wait until the device has finished or run every enqueued slot
        const auto t0 = std::chrono::steady_clock::now();
        int seq = 0, st = kStIter;
        for (long spin = 1;; ++spin) {
            mirror_seq(mh, &seq, &st);
            if (seq > 0 && (st == kStDone || seq >= n_enq)) break;
            if ((spin & 255) == 0) {
                const hipError_t q = hipStreamQuery(s);
                if (q != hipSuccess && q != hipErrorNotReady) {
                    set_error(std::string("device error during GMRES: ") + hipGetErrorString(q));
                    return KFBI_EDEVICE;
                }
                if (q == hipSuccess) {  // stream drained: the mirror must be final
                    mirror_seq(mh, &seq, &st);
                    if (seq > 0 && (st == kStDone || seq >= n_enq)) break;
                    set_error("GMRES control block not published by the device");
                    return KFBI_EDEVICE;
                }
                if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(120)) {
                    set_error("timed out waiting for the GMRES control block");
                    return KFBI_EDEVICE;
                }
            }
        }
        seq_last = seq;
        if (st == kStDone) {
            d->slot_hist[d->slot_pos++ & 3] = seq;
            break;
        }
        want = 4;
    }
    if (d->prof_on) KFBI_TRY(prof_flush(d, seq_last, kTailTag + last_batch));
    *iters_out = mh->iters;
    *rel_out = mh->bnorm > 0 ? mh->resid / mh->bnorm : mh->resid;
    *conv_out = mh->converged;
    *cycles_out = mh->cycles;
    return KFBI_OK;
}

// Replay timing of the control kernel: back-to-back Arnoldi steps on column
// j_r = min(5, last column of the last solve) of the last solve's basis, in
// replay mode (the control block set once to a step at j_r that cannot stop,
// and not advanced by the launches).  The basis columns above j_r, H, the
// rotations, g and vcur are overwritten (every solve starts by rewriting
// them); the density x and the control block are left as the last solve
// ended.
template <class T>
int replay_slot_t(kfbi_domain *d, int reps, double *avg_ms, double *bytes) {
    hipStream_t s = d->stream;
    GmPtrs P = gm_layout(d, 64);
    const int Nb = d->Nb;
    GmCtl c;
    KFBI_HIP(hipMemcpyAsync(&c, P.ctl, sizeof(GmCtl), hipMemcpyDeviceToHost, s));
    KFBI_HIP(hipStreamSynchronize(s));
    const int m = c.m > 1 ? c.m : 2;
    int jr = c.j - 1 < 5 ? c.j - 1 : 5;
    if (jr < 0) jr = 0;
    if (jr > m - 2) jr = m - 2;
    GmCtl r = c;
    r.state = kStIter;
    r.j = jr;
    r.iters = 0;
    r.fixed = 0;
    r.max_iter = 1 << 30;
    r.thresh = -1.0;  // never converged: the step cannot end the cycle
    r.eta = 0.0;
    r.mixed = 0;
    r.slot = 0;
    r.skip64 = 0;
    r.skip32 = 1;
    r.skip_tail = 1;
    KFBI_HIP(hipMemcpyAsync(P.ctl, &r, sizeof(GmCtl), hipMemcpyHostToDevice, s));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = KFBI_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = KFBI_EDEVICE;
    const bool was_on = d->prof_on;
    d->prof_on = false;
    if (rc == KFBI_OK) rc = launch_slot<T>(d, P, Nb, m, jr + 1, s, true);  // warm-up
    if (rc == KFBI_OK && hipEventRecord(e0, s) != hipSuccess) rc = KFBI_EDEVICE;
    for (int q = 0; q < reps && rc == KFBI_OK; ++q) rc = launch_slot<T>(d, P, Nb, m, jr + 1, s, true);
    if (rc == KFBI_OK && hipEventRecord(e1, s) != hipSuccess) rc = KFBI_EDEVICE;
    if (rc == KFBI_OK && hipEventSynchronize(e1) != hipSuccess) rc = KFBI_EDEVICE;
    float ms = 0.f;
    if (rc == KFBI_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = KFBI_EDEVICE;
    d->prof_on = was_on;
    // leave the control block as the last solve ended
    if (hipMemcpyAsync(P.ctl, &c, sizeof(GmCtl), hipMemcpyHostToDevice, s) != hipSuccess && rc == KFBI_OK)
        rc = KFBI_EDEVICE;
    if (hipStreamSynchronize(s) != hipSuccess && rc == KFBI_OK) rc = KFBI_EDEVICE;
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (rc != KFBI_OK) {
        set_error("replay of the control kernel failed");
        return rc;
    }
    *avg_ms = (double)ms / reps;
    // the algorithmic bytes of launch_slot's accounting at column jr
    const double es = (double)sizeof(T);
    *bytes = (double)Nb * es + 2.0 * (jr + 1) * Nb * es + 2.0 * Nb * es;
    return KFBI_OK;
}

int replay_slot(kfbi_domain *d, int reps, double *avg_ms, double *bytes) {
    if (!d->gm || !d->mirror_dev) {
        set_error("no device-driven solve has run on this domain");
        return KFBI_EINVAL;
    }
    const bool slots = d->cplx ? slots_supported<cd>(d, 50) : slots_supported<double>(d, 50);
    if (!slots) {
        set_error("the domain does not use the device-driven schedule");
        return KFBI_ENOTSUP;
    }
    return d->cplx ? replay_slot_t<cd>(d, reps, avg_ms, bytes) : replay_slot_t<double>(d, reps, avg_ms, bytes);
}

int helmholtz_solve(kfbi_domain *d, double kre, double kim, const void *f_grid, const void *f_gamma,
                    const void *g_gamma, void *u_grid_out, void *phi_inout, const kfbi_solve_opts *opts,
                    kfbi_solve_stats *stats, int bc, void *trace_out, const GridUpdate *up) {
    kfbi_solve_opts o;
    o.tol = 1e-10;
    o.max_iter = 500;
    o.restart = 50;
    o.fixed_iters = 0;
    o.precision = -1;
    o.flags = 0;
    o.pad = 0;
    o.gamma = 0.0;
    if (opts) {
        if (opts->tol > 0) o.tol = opts->tol;
        if (opts->max_iter > 0) o.max_iter = opts->max_iter;
        if (opts->restart > 0) o.restart = opts->restart;
        o.fixed_iters = opts->fixed_iters;
        o.precision = opts->precision;
        o.flags = opts->flags;
        o.gamma = opts->gamma;
    }
    if (o.restart > 64) {
        set_error("restart length must be at most 64");
        return KFBI_EINVAL;
    }
    if (f_grid && !f_gamma) {
        set_error("f_gamma is required when f_grid is given");
        return KFBI_EINVAL;
    }
    if (d->Nb > kGmThreads * 16) {
        set_error("too many collocation points for the Arnoldi kernel");
        return KFBI_ENOTSUP;
    }
    const int prec = o.precision >= 0 ? o.precision : d->desc.precision;
    if (prec != KFBI_PREC_FP64 && prec != KFBI_PREC_MIXED) {
        set_error("unknown precision mode");
        return KFBI_EINVAL;
    }
    const bool mixed = prec == KFBI_PREC_MIXED;
    const bool rich = (o.flags & KFBI_SOLVE_RICHARDSON) != 0;
    if (rich && mixed) {
        set_error("the Richardson iteration runs in FP64 only");
        return KFBI_ENOTSUP;
    }
    hipStream_t s = d->stream;
    if (!d->ev0) {
        KFBI_HIP(hipEventCreate(&d->ev0));
        KFBI_HIP(hipEventCreate(&d->ev1));
    }
    hipEvent_t e0 = d->ev0, e1 = d->ev1;
    KFBI_HIP(hipEventRecord(e0, s));
    GmPtrs P = gm_layout(d, 64);
    const size_t vb = (size_t)d->Nb * elem_size(d);
    KFBI_TRY(ensure_coefficients(d, kre, kim));
    KFBI_TRY(tune_tridiag(d));
    KFBI_TRY(ensure_operators(d, kre, kim, bc));
    if (bc && (size_t)d->Nb * elem_size(d) > 65536) {
        set_error("the Neumann solve needs Nb <= 8192 (real) or 4096 (complex)");
        return KFBI_ENOTSUP;
    }
    if (bc && !d->op_merged) {
        set_error("the Neumann solve needs the merged operators (a node's edge windows are too far apart)");
        return KFBI_ENOTSUP;
    }
    if (mixed) KFBI_TRY(ensure_coefficients_low(d, kre, kim));
    // b = g - IS(f, 0).U+ (Dirichlet), b = g - IS(f, 0, 0).dU+/dn (Neumann)
    if (f_grid) {
        // the DST of f and the corrections of f alone in one launch; the
        // corrections are kept: the final solve adds those of the density to
        // them (the interface problem is affine in phi)
        KFBI_TRY(dst_rows_dense_corr(d, f_grid, d->rhat, kre, kim, f_gamma, d->corr_f));
        KFBI_TRY(tridiag_solve(d, d->rhat, d->corr_f, d->uhat));
        if (bc) {
            KFBI_TRY(eval_stencil_nodes(d, d->uhat, d->ust));
            KFBI_TRY(extract_boundary_psi_ctl(d, kre, kim, d->ust, f_gamma, nullptr, true, g_gamma, -1.0, P.b,
                                              nullptr));
        } else {
            // stencil values and extraction in one launch
            KFBI_TRY(eval_extract_boundary(d, kre, kim, d->uhat, f_gamma, g_gamma, -1.0, P.b));
        }
    } else {
        KFBI_HIP(hipMemcpyAsync(P.b, g_gamma, vb, hipMemcpyDeviceToDevice, s));
    }
    int iters = 0, conv = 0, cycles = 0;
    double rel = 0.0;
    int st;
    // U = IS(f, phi).U on the grid (gate: null, or the finish flag of the
    // device-driven schedule)
    auto final_solve = [&](const int *gate) -> int {
        bool copied = false;  // phi_inout written by the corrections' launch
        if (bc) KFBI_TRY(compute_corrections_psi_ctl(d, kre, kim, f_gamma, P.x, d->corr, gate));
        else if (d->op_merged && (f_grid != nullptr) == (f_gamma != nullptr)) {
            // corrections of f (from the b-solve) plus the density's, by the
            // merged operator; the same launch copies the density out
            copied = gate && phi_inout;
            KFBI_TRY(corrections_of_density(d, P.x, d->corr, gate, f_grid ? d->corr_f : nullptr,
                                            copied ? phi_inout : nullptr));
        } else KFBI_TRY(compute_corrections_ctl(d, kre, kim, P.x, nullptr, f_gamma, d->corr, gate));
        KFBI_TRY(tridiag_solve_ctl(d, f_grid ? d->rhat : nullptr, d->corr, d->uhat, gate));
        // the inverse transform also makes the caller's state update, if any
        if (u_grid_out) KFBI_TRY(idst_rows_dense_ctl(d, d->uhat, u_grid_out, gate, up));
        if (bc && trace_out) {
            // U+ of the solution at the collocation points (the trace of u)
            KFBI_TRY(eval_stencil_nodes_ctl(d, d->uhat, d->ust, gate));
            KFBI_TRY(extract_boundary_psi_ctl(d, kre, kim, d->ust, f_gamma, P.x, false, nullptr, 1.0, trace_out,
                                              gate));
        }
        if (phi_inout && !copied) {
            if (gate) {
                const int n = (int)(vb / sizeof(double));
                k_copy_gated<double><<<(n + 255) / 256, 256, 0, s>>>(n, (double *)phi_inout, (const double *)P.x,
                                                                      gate);
                KFBI_CHECK_LAUNCH();
            } else {
                KFBI_HIP(hipMemcpyAsync(phi_inout, P.x, vb, hipMemcpyDeviceToDevice, s));
            }
        }
        return KFBI_OK;
    };
    const bool slots = d->cplx ? slots_supported<cd>(d, o.restart) : slots_supported<double>(d, o.restart);
    if (rich && !slots) {
        set_error("the Richardson iteration needs the device-driven schedule (merged operators)");
        return KFBI_ENOTSUP;
    }
    if (slots) {
        // the start vector is placed by the schedule's first kernel
        if (d->cplx) st = gmres_run_slots<cd>(d, P, phi_inout, o, mixed, final_solve, &iters, &rel, &conv, &cycles);
        else st = gmres_run_slots<double>(d, P, phi_inout, o, mixed, final_solve, &iters, &rel, &conv, &cycles);
        if (st != KFBI_OK) return st;
    } else {
        if (phi_inout) KFBI_HIP(hipMemcpyAsync(P.x, phi_inout, vb, hipMemcpyDeviceToDevice, s));
        else KFBI_HIP(hipMemsetAsync(P.x, 0, vb, s));
        if (d->cplx) st = gmres_run<cd>(d, kre, kim, P, o, mixed, &iters, &rel, &conv, &cycles);
        else st = gmres_run<double>(d, kre, kim, P, o, mixed, &iters, &rel, &conv, &cycles);
        if (st != KFBI_OK) return st;
        KFBI_TRY(final_solve(nullptr));
    }
    KFBI_HIP(hipEventRecord(e1, s));
    float ms = -1.f;
    if (!(o.flags & KFBI_SOLVE_ASYNC)) {
        KFBI_HIP(hipEventSynchronize(e1));
        KFBI_HIP(hipEventElapsedTime(&ms, e0, e1));
    }
    if (stats) {
        stats->iters = iters;
        stats->converged = conv;
        stats->rel_resid = rel;
        stats->refinements = mixed ? cycles : 0;
        stats->device_ms = ms;
    }
    const bool fixed = o.fixed_iters > 0;
    if (!conv && !fixed) {
        set_error(rich ? "the Richardson iteration reached max_iter before the tolerance"
                       : "GMRES reached max_iter before the tolerance");
        return KFBI_ENOCONV;
    }
    return KFBI_OK;
}

// ---------------------------------------------------------------------------
// Batched solves: many real domains advance through the same launches.  Each
// member keeps its own device-driven GMRES state (control block, gates,
// mirror); a batched kernel runs every member's blocks and each block obeys
// its own member's gate, so members that finish early cost only the early
// exit of their blocks.
// ---------------------------------------------------------------------------
namespace {

struct CopyArgs {
    double *dst;
    const double *src;  // null: zero
    int n;
    const int *done;
};

__device__ void copy_body(const CopyArgs &A, int blk) {
    if (A.done && *A.done) return;
    const int i = blk * blockDim.x + threadIdx.x;
    if (i < A.n) A.dst[i] = A.src ? A.src[i] : 0.0;
}

struct FinalArgs {
    int *skip_tail;
};

__global__ __launch_bounds__(256) void kb_copy(const CopyArgs *__restrict__ A, const BlkMap *__restrict__ map) {
    const BlkMap e = map[blockIdx.x];
    copy_body(A[e.inst], e.local);
}

// a member whose final solve has just run (skip_tail 0) is marked done (2),
// so later rounds of the same solve skip it
__global__ void kb_final(const FinalArgs *__restrict__ A, int n) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n && *A[q].skip_tail == 0) *A[q].skip_tail = 2;
}

template <class T>
__global__ __launch_bounds__(kGmThreads) void kb_gm_init(const GmInitArgs<T> *__restrict__ A) {
    gm_init_body(A[blockIdx.x], 0);
}

template <class T, int EPT>
__global__ __launch_bounds__(kGmThreads) void kb_gm_slot(const SlotArgs<T> *__restrict__ A) {
    gm_slot_body<T, EPT>(A[blockIdx.x], 0);
}

// argument arrays of one batched solve, one entry per member each
enum {
    kUDstF = 0, kUCorrB, kUTriB, kUErowB, kUExtB, kUCopyX, kUInit,
    kUCorrPhi64, kUTri64, kUErow64, kUExm64, kUCorrPhi32, kUTri32, kUErow32, kUExm32, kUSlot,
    kUCorrF, kUTriF, kUIdst, kUZero, kUCopyF, kUFinal, kUses
};

}  // namespace

// members of equal M share the tridiagonal launches: one workgroup map per
// choice of 1, 2, 4 or 8 modes per workgroup, and the shape in use for the
// sparse FP64, dense-input FP64 and sparse FP32 solves
struct BatchClass {
    int M;
    std::vector<int> members;
    int map_mb[4], blocks_mb[4];
    int map_erow, blocks_erow;
    BatchTriShape shape[3];
    bool tuned[3];
    double us[3];
};

inline int mb_log2(int mb) { return mb >= 8 ? 3 : mb >= 4 ? 2 : mb >= 2 ? 1 : 0; }

}  // namespace kfbi

struct kfbi_batch {
    std::vector<kfbi_domain *> doms;
    hipStream_t stream = nullptr;
    bool cplx = false;  // every member complex (else every member real)
    // workgroup maps, one array for all kinds and classes
    kfbi::BlkMap *d_map = nullptr;
    int map_off[kfbi::kBaKinds] = {}, map_blocks[kfbi::kBaKinds] = {};
    std::vector<kfbi::BatchClass> classes;
    // argument staging
    char *h_args = nullptr, *d_args = nullptr;
    size_t use_off[kfbi::kUses] = {}, use_size[kfbi::kUses] = {}, args_bytes = 0;
    int slot_hist[4] = {0, 0, 0, 0};  // slots of the last four batched solves
    int slot_pos = 0;
    int nb_max = 0, m_lds = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int *d_one = nullptr;  // a device word holding 1: the gate of members not solved in a call
};

namespace kfbi {

void batch_destroy(kfbi_batch *b) {
    if (!b) return;
    if (b->stream) hipStreamSynchronize(b->stream);
    if (b->d_map) hipFree(b->d_map);
    if (b->d_args) hipFree(b->d_args);
    if (b->d_one) hipFree(b->d_one);
    if (b->h_args) hipHostFree(b->h_args);
    if (b->ev0) hipEventDestroy(b->ev0);
    if (b->ev1) hipEventDestroy(b->ev1);
    delete b;
}

int batch_create(kfbi_domain *const *doms, int n, kfbi_batch **out) {
    if (!doms || n < 1 || !out) { set_error("null argument or empty batch"); return KFBI_EINVAL; }
    *out = nullptr;
    if (!doms[0]) { set_error("null domain in batch"); return KFBI_EINVAL; }
    kfbi_batch *b = new kfbi_batch();
    b->stream = doms[0]->stream;
    b->cplx = doms[0]->cplx;
    for (int q = 0; q < n; ++q) {
        kfbi_domain *d = doms[q];
        if (!d) { batch_destroy(b); set_error("null domain in batch"); return KFBI_EINVAL; }
        if (d->cplx != b->cplx) {
            batch_destroy(b);
            set_error("batch members must share one scalar type (all real or all complex)");
            return KFBI_EINVAL;
        }
        if (d->stream != b->stream) {
            batch_destroy(b);
            set_error("batch members must share one stream");
            return KFBI_EINVAL;
        }
        if ((size_t)d->Nb * elem_size(d) > 65536) {
            batch_destroy(b);
            set_error("batch members need Nb <= 8192 (real) or 4096 (complex)");
            return KFBI_ENOTSUP;
        }
        if (d->M < 64) {
            // the row-wise stencil evaluation holds a row of 64 KR modes in
            // registers, KR >= 1
            batch_destroy(b);
            set_error("batch members need M >= 64");
            return KFBI_ENOTSUP;
        }
        if (d->erow_blk_max > kErowCols) {
            batch_destroy(b);
            set_error("batch member with too many stencil nodes on consecutive rows");
            return KFBI_ENOTSUP;
        }
        b->doms.push_back(d);
        b->nb_max = std::max(b->nb_max, d->Nb);
    }
    // workgroup maps: per kind over all members (the tridiagonal kinds per
    // class of equal M, in XCD tile order inside the kernel)
    std::vector<BlkMap> map;
    const int kinds[] = {kBaDst, kBaZero, kBaExm, kBaCorrPhi, kBaCorr, kBaExt, kBaCopy};
    for (int kind : kinds) {
        b->map_off[kind] = (int)map.size();
        for (int q = 0; q < n; ++q) {
            int nbk;
            if (kind == kBaCorr || kind == kBaExt) nbk = batch_blocks_iface(doms[q], kind);
            else if (kind == kBaCopy) nbk = ((doms[q]->cplx ? 2 : 1) * doms[q]->Nb + 255) / 256;  // doubles
            else nbk = batch_blocks(doms[q], kind);
            for (int l = 0; l < nbk; ++l) map.push_back(BlkMap{q, l});
        }
        b->map_blocks[kind] = (int)map.size() - b->map_off[kind];
    }
    std::vector<int> Ms;
    for (int q = 0; q < n; ++q)
        if (std::find(Ms.begin(), Ms.end(), doms[q]->M) == Ms.end()) Ms.push_back(doms[q]->M);
    std::sort(Ms.begin(), Ms.end());
    for (int M : Ms) {
        BatchClass C;
        C.M = M;
        for (int q = 0; q < n; ++q)
            if (doms[q]->M == M) C.members.push_back(q);
        std::vector<kfbi_domain *> cd;
        for (int q : C.members) cd.push_back(doms[q]);
        for (int kind = 0; kind < 3; ++kind) {
            const int st = batch_tri_shape(cd.data(), (int)cd.size(), true, kind == 2, &C.shape[kind]);
            if (st != KFBI_OK) { batch_destroy(b); return st; }
            C.shape[kind].dense = kind == 1;
            C.tuned[kind] = false;
            C.us[kind] = -1.0;
        }
        for (int lm = 0; lm < 4; ++lm) {
            C.map_mb[lm] = (int)map.size();
            for (int q : C.members)
                for (int l = 0; l < batch_tri_blocks(doms[q], 1 << lm); ++l) map.push_back(BlkMap{q, l});
            C.blocks_mb[lm] = (int)map.size() - C.map_mb[lm];
        }
        C.map_erow = (int)map.size();
        for (int q : C.members)
            for (int l = 0; l < batch_blocks(doms[q], kBaErow64); ++l) map.push_back(BlkMap{q, l});
        C.blocks_erow = (int)map.size() - C.map_erow;
        b->classes.push_back(C);
    }
    // argument arrays
    auto use_size = [&](int u) -> size_t {
        switch (u) {
            case kUDstF: case kUIdst: return batch_args_size(kBaDst, b->cplx);
            case kUZero: return batch_args_size(kBaZero, b->cplx);
            case kUCorrB: return batch_args_size_iface(kBaCorr, b->cplx);
            case kUCorrF: return batch_args_size(kBaCorrPhi, b->cplx);
            case kUExtB: return batch_args_size_iface(kBaExt, b->cplx);
            case kUTriB: case kUTriF: case kUTri64: return batch_args_size(kBaTri64, b->cplx);
            case kUTri32: return batch_args_size(kBaTri32, b->cplx);
            case kUErowB: case kUErow64: return batch_args_size(kBaErow64, b->cplx);
            case kUErow32: return batch_args_size(kBaErow32, b->cplx);
            case kUExm64: case kUExm32: return batch_args_size(kBaExm, b->cplx);
            case kUCorrPhi64: case kUCorrPhi32: return batch_args_size(kBaCorrPhi, b->cplx);
            case kUCopyX: case kUCopyF: return sizeof(CopyArgs);
            case kUInit: return b->cplx ? sizeof(GmInitArgs<cd>) : sizeof(GmInitArgs<double>);
            case kUSlot: return b->cplx ? sizeof(SlotArgs<cd>) : sizeof(SlotArgs<double>);
            case kUFinal: return sizeof(FinalArgs);
            default: return 0;
        }
    };
    size_t off = 0;
    for (int u = 0; u < kUses; ++u) {
        b->use_size[u] = use_size(u);
        b->use_off[u] = off;
        off += ((b->use_size[u] * n) + 255) & ~(size_t)255;
    }
    b->args_bytes = off;
    if (hipHostMalloc((void **)&b->h_args, off, hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void **)&b->d_args, off) != hipSuccess ||
        hipMalloc((void **)&b->d_map, map.size() * sizeof(BlkMap)) != hipSuccess ||
        hipMalloc((void **)&b->d_one, sizeof(int)) != hipSuccess) {
        batch_destroy(b);
        set_error("out of device memory for the batch tables");
        return KFBI_ENOMEM;
    }
    static const int one = 1;
    if (hipMemcpyAsync(b->d_map, map.data(), map.size() * sizeof(BlkMap), hipMemcpyHostToDevice, b->stream) !=
            hipSuccess ||
        hipMemcpyAsync(b->d_one, &one, sizeof(int), hipMemcpyHostToDevice, b->stream) != hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess) {
        batch_destroy(b);
        set_error("copy of the batch tables failed");
        return KFBI_EDEVICE;
    }
    if (hipEventCreate(&b->ev0) != hipSuccess || hipEventCreate(&b->ev1) != hipSuccess) {
        batch_destroy(b);
        set_error("hipEventCreate failed");
        return KFBI_EDEVICE;
    }
    *out = b;
    return KFBI_OK;
}

// microseconds per launch of one class's tridiagonal solves in shape S: one
// launch to warm up, one to size the run, then about 2 ms of launches
int tune_time(kfbi_batch *b, int kind, const void *args, const BatchClass &C, const BatchTriShape &S, double *us) {
    hipStream_t s = b->stream;
    const int lm = mb_log2(S.mb);
    auto go = [&]() {
        return batch_launch(kind, args, b->d_map + C.map_mb[lm], C.blocks_mb[lm], C.M, &S, s, b->cplx);
    };
    KFBI_TRY(go());
    float ms = 0.f;
    KFBI_HIP(hipEventRecord(b->ev0, s));
    KFBI_TRY(go());
    KFBI_HIP(hipEventRecord(b->ev1, s));
    KFBI_HIP(hipEventSynchronize(b->ev1));
    KFBI_HIP(hipEventElapsedTime(&ms, b->ev0, b->ev1));
    const int reps = std::min(20, std::max(2, (int)(2.0 / std::max(ms, 1e-3f)) + 1));
    KFBI_HIP(hipEventRecord(b->ev0, s));
    for (int r = 0; r < reps; ++r) KFBI_TRY(go());
    KFBI_HIP(hipEventRecord(b->ev1, s));
    KFBI_HIP(hipEventSynchronize(b->ev1));
    KFBI_HIP(hipEventElapsedTime(&ms, b->ev0, b->ev1));
    *us = 1e3 * ms / reps;
    return KFBI_OK;
}

// Times the tridiagonal launch shapes of every class once per precision and
// keeps the fastest.  Only shapes with 64-lane mode groups (1, 2 or 4 modes
// per workgroup; the tile kernel, and for sparse input also the register-row
// kernel) are candidates: for a given mode they run the same operations in
// the same order, so the choice never changes the values.
// Inputs are the members' own tables with the scratch right-hand sides
// cleared; the launches write only the scratch transforms.
int batch_tune_run(kfbi_batch *b, bool low, char *d_buf, const uint8_t *active) {
    const int n = (int)b->doms.size();
    const size_t as = batch_args_size(low ? kBaTri32 : kBaTri64, b->cplx);
    for (auto &C : b->classes) {
        std::vector<kfbi_domain *> cd;
        bool any = false;
        for (int q : C.members) {
            cd.push_back(b->doms[q]);
            any = any || !active || active[q];
        }
        if (!any) continue;  // timed once some member of the class is solved
        const int kinds_hi[] = {0, 1}, kinds_lo[] = {2};
        const int *kinds = low ? kinds_lo : kinds_hi;
        const int nk = low ? 1 : 2;
        for (int ik = 0; ik < nk; ++ik) {
            const int kind = kinds[ik];
            if (C.tuned[kind] || C.shape[kind].mb > 4) continue;
            const void *args = d_buf + (kind == 1 ? (size_t)n * as : 0);
            BatchTriShape best = C.shape[kind];
            double best_us = 1e300;
            const int pref = tri_kernel_pref();
            for (int rows = 0; rows < 2; ++rows) {
                if (pref >= 0 && rows != pref) continue;
                for (int mb : {1, 2, 4, 8}) {
                    if (mb == 8 && !rows) continue;  // 32-lane groups: other values
                    if (tri_mb_pref() > 0 && mb != tri_mb_pref()) continue;
                    for (int stage : {0, 1}) {
                        if (tri_stage_pref() >= 0 && stage != tri_stage_pref()) continue;
                        BatchTriShape S;
                        if (batch_tri_shape(cd.data(), (int)cd.size(), true, low, &S, mb, stage, rows != 0) != KFBI_OK)
                            continue;
                        S.dense = rows != 0 && kind == 1;
                        double us = 0.0;
                        KFBI_TRY(tune_time(b, low ? kBaTri32 : kBaTri64, args, C, S, &us));
                        if (us < best_us) {
                            best_us = us;
                            best = S;
                        }
                    }
                }
            }
            C.shape[kind] = best;
            C.us[kind] = best_us;
            C.tuned[kind] = true;
        }
    }
    return KFBI_OK;
}

int batch_tune(kfbi_batch *b, bool low, const uint8_t *active) {
    bool need = false;
    for (auto &C : b->classes)
        for (int kind : {0, 1, 2})
            if ((kind == 2) == low && !C.tuned[kind] && C.shape[kind].mb <= 4) need = true;
    if (!need) return KFBI_OK;
    const int n = (int)b->doms.size();
    hipStream_t s = b->stream;
    const size_t as = batch_args_size(low ? kBaTri32 : kBaTri64, b->cplx);
    std::vector<char> h(2 * as * n);
    for (int q = 0; q < n; ++q) {
        kfbi_domain *d = b->doms[q];
        const int nn = d->M - 1;
        // members not solved in this call may lack their coefficients: gated off
        const int *one = (!active || active[q]) ? nullptr : b->d_one;
        if (!one) {
            KFBI_HIP(hipMemsetAsync(d->corr, 0, (size_t)d->n_irr * elem_size(d), s));
            KFBI_HIP(hipMemsetAsync(d->rhat, 0, (size_t)nn * nn * elem_size(d), s));
        }
        batch_fill_tri(d, nullptr, d->corr, low ? d->uhat32 : d->uhat, one, low, h.data() + (size_t)q * as);
        if (!low) batch_fill_tri(d, d->rhat, d->corr, d->uhat, one, false, h.data() + (size_t)(n + q) * as);
    }
    char *d_buf = nullptr;
    KFBI_HIP(hipMalloc((void **)&d_buf, h.size()));
    int st = hipMemcpyAsync(d_buf, h.data(), h.size(), hipMemcpyHostToDevice, s) == hipSuccess ? KFBI_OK
                                                                                                 : KFBI_EDEVICE;
    if (st != KFBI_OK) set_error("copy of the tuning arguments failed");
    if (st == KFBI_OK) st = batch_tune_run(b, low, d_buf, active);
    const bool synced = hipStreamSynchronize(s) == hipSuccess;
    hipFree(d_buf);
    if (st == KFBI_OK && !synced) {
        set_error("stream failed while tuning the batch");
        st = KFBI_EDEVICE;
    }
    return st;
}

int batch_size(const kfbi_batch *b) { return (int)b->doms.size(); }
kfbi_domain *batch_domain(const kfbi_batch *b, int q) { return b->doms[q]; }

int batch_tuning(const kfbi_batch *b, int cap, int32_t *rows, double *us, int32_t *n_rows) {
    if (!b || !n_rows || cap < 0 || (cap > 0 && !rows)) { set_error("null argument"); return KFBI_EINVAL; }
    int r = 0;
    for (const auto &C : b->classes)
        for (int kind = 0; kind < 3; ++kind, ++r) {
            if (r >= cap) continue;
            int32_t *o = rows + 6 * r;
            o[0] = C.M;
            o[1] = kind;
            o[2] = C.shape[kind].mb;
            o[3] = C.shape[kind].stage ? 1 : 0;
            o[4] = C.tuned[kind] ? 1 : 0;
            o[5] = C.shape[kind].rows ? 1 : 0;
            if (us) us[r] = C.tuned[kind] ? C.us[kind] : -1.0;
        }
    *n_rows = r;
    return KFBI_OK;
}

namespace {
template <class T>
int batch_helmholtz_t(kfbi_batch *b, const double *kappa, const double *kappa_im, const void *const *f_grid,
                      const void *const *f_gamma, const void *const *g_gamma, void *const *u_out,
                      void *const *phi_inout, const kfbi_solve_opts *opts, kfbi_solve_stats *stats,
                      const uint8_t *active) {
    auto kim = [&](int q) { return kappa_im ? kappa_im[q] : 0.0; };
    const bool cplx = b->cplx;
    // a complex element moves as two doubles in the density copies
    const int cw = cplx ? 2 : 1;
    const int n = (int)b->doms.size();
    auto on = [&](int q) { return !active || active[q] != 0; };
    int n_on = 0;
    for (int q = 0; q < n; ++q) n_on += on(q) ? 1 : 0;
    if (stats)
        for (int q = 0; q < n; ++q) stats[q] = kfbi_solve_stats{0, 1, 0.0, 0, 0, 0.0};
    if (n_on == 0) return KFBI_OK;
    kfbi_solve_opts o;
    o.tol = 1e-10;
    o.max_iter = 500;
    o.restart = 50;
    o.fixed_iters = 0;
    o.precision = -1;
    o.flags = 0;
    o.pad = 0;
    o.gamma = 0.0;
    if (opts) {
        if (opts->tol > 0) o.tol = opts->tol;
        if (opts->max_iter > 0) o.max_iter = opts->max_iter;
        if (opts->restart > 0) o.restart = opts->restart;
        o.fixed_iters = opts->fixed_iters;
        o.precision = opts->precision;
        o.flags = opts->flags;
        o.gamma = opts->gamma;
    }
    if (o.restart > 64) { set_error("restart length must be at most 64"); return KFBI_EINVAL; }
    if (o.flags & KFBI_SOLVE_RICHARDSON) { set_error("batched solves use GMRES"); return KFBI_ENOTSUP; }
    const bool mixed = (o.precision >= 0 ? o.precision : b->doms[0]->desc.precision) == KFBI_PREC_MIXED;
    hipStream_t s = b->stream;
    // per-member setup: coefficients and operators for this kappa
    for (int q = 0; q < n; ++q) {
        kfbi_domain *d = b->doms[q];
        if (!on(q)) continue;
        if (!f_grid[q] || !f_gamma[q] || !g_gamma[q]) { set_error("null member array"); return KFBI_EINVAL; }
        KFBI_TRY(ensure_coefficients(d, kappa[q], kim(q)));
        KFBI_TRY(ensure_operators(d, kappa[q], kim(q)));
        if (mixed) KFBI_TRY(ensure_coefficients_low(d, kappa[q], kim(q)));
        if (!slots_supported<T>(d, o.restart)) {
            set_error("batch member without the merged operators or too large for the control kernel");
            return KFBI_ENOTSUP;
        }
        if (!d->mirror_host) {
            KFBI_HIP(hipHostMalloc(&d->mirror_host, sizeof(GmMirror), hipHostMallocMapped | hipHostMallocCoherent));
            memset(d->mirror_host, 0, sizeof(GmMirror));
            KFBI_HIP(hipHostGetDevicePointer(&d->mirror_dev, d->mirror_host, 0));
        }
    }
    if (!(o.flags & KFBI_BATCH_NO_TUNE)) {
        KFBI_TRY(batch_tune(b, false, active));
        if (mixed) KFBI_TRY(batch_tune(b, true, active));
    }
    // argument blocks
    size_t slot_lds_max = 0;
    for (int q = 0; q < n; ++q) {
        kfbi_domain *d = b->doms[q];
        GmPtrs P = gm_layout(d, 64);
        // a member not solved in this call has every gate on the word that holds 1
        const int *one = on(q) ? nullptr : b->d_one;
        const int *skip64 = one ? one : &P.ctl->skip64, *skip32 = one ? one : &P.ctl->skip32,
                  *skip_tail = one ? one : &P.ctl->skip_tail;
        auto at = [&](int u) { return b->h_args + b->use_off[u] + (size_t)q * b->use_size[u]; };
        batch_fill_dst(d, f_grid[q], true, true, d->rhat, false, 1.0, one, at(kUDstF));
        batch_fill_corr(d, kappa[q], kim(q), nullptr, f_gamma[q], d->corr_f, one, at(kUCorrB));
        batch_fill_tri(d, d->rhat, d->corr_f, d->uhat, one, false, at(kUTriB));
        batch_fill_erow(d, d->uhat, d->ust, one, false, at(kUErowB));
        batch_fill_ext(d, kappa[q], kim(q), d->ust, nullptr, f_gamma[q], g_gamma[q], -1.0, P.b, one, at(kUExtB));
        *(CopyArgs *)at(kUCopyX) = CopyArgs{(double *)P.x, phi_inout ? (const double *)phi_inout[q] : nullptr,
                                            cw * d->Nb, one};
        GmInitArgs<T> ia = gm_init_args<T>(P, d->Nb, o, mixed, P.x);
        ia.off = one;
        *(GmInitArgs<T> *)at(kUInit) = ia;
        batch_fill_corr_phi(d, P.vcur, d->corr, skip64, at(kUCorrPhi64));
        batch_fill_tri(d, nullptr, d->corr, d->uhat, skip64, false, at(kUTri64));
        batch_fill_erow(d, d->uhat, d->ust, skip64, false, at(kUErow64));
        batch_fill_exm(d, d->ust, P.vcur, P.r, skip64, at(kUExm64));
        batch_fill_corr_phi(d, P.vcur, d->corr, skip32, at(kUCorrPhi32));
        batch_fill_tri(d, nullptr, d->corr, d->uhat32, skip32, true, at(kUTri32));
        batch_fill_erow(d, d->uhat32, d->ust, skip32, true, at(kUErow32));
        batch_fill_exm(d, d->ust, P.vcur, P.r, skip32, at(kUExm32));
        int nvl;
        const size_t lds = slot_lds<T>(d->Nb, o.restart, &nvl);
        slot_lds_max = std::max(slot_lds_max, lds);
        SlotArgs<T> sa = slot_args<T>(P, (GmMirror *)d->mirror_dev, d->Nb, o.restart, nvl);
        sa.off = one;
        *(SlotArgs<T> *)at(kUSlot) = sa;
        batch_fill_corr_phi(d, P.x, d->corr, skip_tail, at(kUCorrF), d->corr_f);
        batch_fill_tri(d, d->rhat, d->corr, d->uhat, skip_tail, false, at(kUTriF));
        void *uo = u_out ? u_out[q] : nullptr;
        batch_fill_dst(d, d->uhat, false, false, uo, true, 2.0 / d->M, skip_tail, at(kUIdst));
        batch_fill_zero(d, uo, skip_tail, at(kUZero));
        *(CopyArgs *)at(kUCopyF) = CopyArgs{phi_inout ? (double *)phi_inout[q] : nullptr, (const double *)P.x,
                                            cw * d->Nb, skip_tail};
        *(FinalArgs *)at(kUFinal) = FinalArgs{one ? b->d_one : &P.ctl->skip_tail};
        if (on(q)) __atomic_store_n(&((GmMirror *)d->mirror_host)->seq, 0, __ATOMIC_RELEASE);
    }
    // every member keeps the layout of its own single solve (its own number
    // of staged basis vectors, so the same Gram-Schmidt code path and the
    // same rounding); the launch's dynamic LDS holds the largest layout
    KFBI_HIP(hipEventRecord(b->ev0, s));
    KFBI_HIP(hipMemcpyAsync(b->d_args, b->h_args, b->args_bytes, hipMemcpyHostToDevice, s));
    auto dargs = [&](int u) { return (const void *)(b->d_args + b->use_off[u]); };
    auto mapk = [&](int kind) { return b->d_map + b->map_off[kind]; };
    auto launch = [&](int kind, int use) -> int {
        return batch_launch(kind, dargs(use), mapk(kind), b->map_blocks[kind], 0, nullptr, s, cplx);
    };
    // DST launches: LDS for the largest grid (each block uses its own M)
    int m_max = 0;
    for (auto *d : b->doms) m_max = std::max(m_max, d->M);
    auto launch_dst = [&](int use) -> int {
        return batch_launch(kBaDst, dargs(use), mapk(kBaDst), b->map_blocks[kBaDst], m_max, nullptr, s, cplx);
    };
    // stencil evaluation per class of equal M (register rows sized to M)
    auto launch_erow = [&](int use, bool low) -> int {
        for (auto &C : b->classes)
            KFBI_TRY(batch_launch(low ? kBaErow32 : kBaErow64, dargs(use), b->d_map + C.map_erow, C.blocks_erow, C.M,
                                  nullptr, s, cplx));
        return KFBI_OK;
    };
    auto launch_tri = [&](int use, bool low, bool dense) -> int {
        for (auto &C : b->classes) {
            const BatchTriShape &S = C.shape[low ? 2 : (dense ? 1 : 0)];
            const int lm = mb_log2(S.mb);
            KFBI_TRY(batch_launch(low ? kBaTri32 : kBaTri64, dargs(use), b->d_map + C.map_mb[lm], C.blocks_mb[lm],
                                  C.M, &S, s, cplx));
        }
        return KFBI_OK;
    };
    // b-solve for every member
    KFBI_TRY(launch_dst(kUDstF));
    KFBI_TRY(batch_launch_iface(kBaCorr, dargs(kUCorrB), mapk(kBaCorr), b->map_blocks[kBaCorr], s, cplx));
    KFBI_TRY(launch_tri(kUTriB, false, true));
    KFBI_TRY(launch_erow(kUErowB, false));
    KFBI_TRY(batch_launch_iface(kBaExt, dargs(kUExtB), mapk(kBaExt), b->map_blocks[kBaExt], s, cplx));
    kb_copy<<<b->map_blocks[kBaCopy], 256, 0, s>>>((const CopyArgs *)dargs(kUCopyX), mapk(kBaCopy));
    KFBI_CHECK_LAUNCH();
    kb_gm_init<T><<<n, kGmThreads, 0, s>>>((const GmInitArgs<T> *)dargs(kUInit));
    KFBI_CHECK_LAUNCH();
    // slots until every member has finished
    const int ept = (b->nb_max + kGmThreads - 1) / kGmThreads;
    // first batch: the most slots any of the last four batched solves took
    // (as for single domains)
    int want = 0;
    for (int q = 0; q < 4; ++q) want = std::max(want, b->slot_hist[q]);
    if (want == 0) want = o.fixed_iters > 0 ? o.fixed_iters + 2 : 16;
    int n_enq = 0;
    for (;;) {
        for (int c = 0; c < want; ++c) {
            KFBI_TRY(launch(kBaCorrPhi, kUCorrPhi64));
            KFBI_TRY(launch_tri(kUTri64, false, false));
            KFBI_TRY(launch_erow(kUErow64, false));
            KFBI_TRY(launch(kBaExm, kUExm64));
            if (mixed) {
                KFBI_TRY(launch(kBaCorrPhi, kUCorrPhi32));
                KFBI_TRY(launch_tri(kUTri32, true, false));
                KFBI_TRY(launch_erow(kUErow32, true));
                KFBI_TRY(launch(kBaExm, kUExm32));
            }
            const SlotArgs<T> *SA = (const SlotArgs<T> *)dargs(kUSlot);
            if (ept <= 1) kb_gm_slot<T, 1><<<n, kGmThreads, slot_lds_max, s>>>(SA);
            else if (ept <= 2) kb_gm_slot<T, 2><<<n, kGmThreads, slot_lds_max, s>>>(SA);
            else if (ept <= 4) kb_gm_slot<T, 4><<<n, kGmThreads, slot_lds_max, s>>>(SA);
            else if (ept <= 8) kb_gm_slot<T, 8><<<n, kGmThreads, slot_lds_max, s>>>(SA);
            else kb_gm_slot<T, 16><<<n, kGmThreads, slot_lds_max, s>>>(SA);
            KFBI_CHECK_LAUNCH();
        }
        n_enq += want;
        // final solve of the members that have finished (gated per member)
        KFBI_TRY(launch(kBaCorrPhi, kUCorrF));
        KFBI_TRY(launch_tri(kUTriF, false, true));
        if (u_out) {
            KFBI_TRY(launch_dst(kUIdst));
            KFBI_TRY(launch(kBaZero, kUZero));
        }
        if (phi_inout) {
            kb_copy<<<b->map_blocks[kBaCopy], 256, 0, s>>>((const CopyArgs *)dargs(kUCopyF), mapk(kBaCopy));
            KFBI_CHECK_LAUNCH();
        }
        kb_final<<<(n + 255) / 256, 256, 0, s>>>((const FinalArgs *)dargs(kUFinal), n);
        KFBI_CHECK_LAUNCH();
        // wait until every member has finished or run every enqueued slot
        const auto t0 = std::chrono::steady_clock::now();
        bool all_done = true;
        for (long spin = 1;; ++spin) {
            all_done = true;
            bool settled = true;
            for (int q = 0; q < n; ++q) {
                if (!on(q)) continue;
                GmMirror *mh = (GmMirror *)b->doms[q]->mirror_host;
                int seq, st;
                mirror_seq(mh, &seq, &st);
                const bool done = seq > 0 && st == kStDone;
                if (!done) all_done = false;
                if (!(done || seq >= n_enq)) settled = false;
            }
            if (settled) break;
            if ((spin & 255) == 0) {
                const hipError_t qe = hipStreamQuery(s);
                if (qe != hipSuccess && qe != hipErrorNotReady) {
                    set_error(std::string("device error during batched GMRES: ") + hipGetErrorString(qe));
                    return KFBI_EDEVICE;
                }
                if (qe == hipSuccess) {
                    // drained: one more look at the mirrors, then give up
                    bool ok = true;
                    for (int q = 0; q < n; ++q) {
                        if (!on(q)) continue;
                        GmMirror *mh = (GmMirror *)b->doms[q]->mirror_host;
                        int seq, st;
                        mirror_seq(mh, &seq, &st);
                        if (!((seq > 0 && st == kStDone) || seq >= n_enq)) ok = false;
                    }
                    if (ok) continue;
                    set_error("batched GMRES control blocks not published by the device");
                    return KFBI_EDEVICE;
                }
                if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(300)) {
                    set_error("timed out waiting for the batched GMRES control blocks");
                    return KFBI_EDEVICE;
                }
            }
        }
        if (all_done) break;
        want = 4;
    }
    int max_seq = 0, st = KFBI_OK;
    for (int q = 0; q < n; ++q) {
        if (!on(q)) continue;
        GmMirror *mh = (GmMirror *)b->doms[q]->mirror_host;
        int seq_q, st_q;
        mirror_seq(mh, &seq_q, &st_q);
        max_seq = std::max(max_seq, seq_q);
        if (stats) {
            stats[q].iters = mh->iters;
            stats[q].converged = mh->converged;
            stats[q].rel_resid = mh->bnorm > 0 ? mh->resid / mh->bnorm : mh->resid;
            stats[q].refinements = mixed ? mh->cycles : 0;
            stats[q].pad = 0;
            stats[q].device_ms = -1.0;
        }
        if (!mh->converged && o.fixed_iters <= 0) st = KFBI_ENOCONV;
    }
    b->slot_hist[b->slot_pos++ & 3] = max_seq;
    KFBI_HIP(hipEventRecord(b->ev1, s));
    if (!(o.flags & KFBI_SOLVE_ASYNC)) {
        KFBI_HIP(hipEventSynchronize(b->ev1));
        float ms = 0.f;
        KFBI_HIP(hipEventElapsedTime(&ms, b->ev0, b->ev1));
        if (stats)
            for (int q = 0; q < n; ++q)
                if (on(q)) stats[q].device_ms = ms;
    }
    if (st == KFBI_ENOCONV) set_error("GMRES reached max_iter before the tolerance for a batch member");
    return st;
}
}  // namespace

int batch_helmholtz(kfbi_batch *b, const double *kappa, const double *kappa_im, const void *const *f_grid,
                    const void *const *f_gamma, const void *const *g_gamma, void *const *u_out,
                    void *const *phi_inout, const kfbi_solve_opts *opts, kfbi_solve_stats *stats,
                    const uint8_t *active) {
    if (!b || !kappa || !f_grid || !f_gamma || !g_gamma) { set_error("null argument"); return KFBI_EINVAL; }
    if (kappa_im && !b->cplx)
        for (int q = 0; q < (int)b->doms.size(); ++q)
            if (kappa_im[q] != 0.0 && (!active || active[q])) {
                set_error("complex kappa needs a batch of complex domains");
                return KFBI_EINVAL;
            }
    if (b->cplx)
        return batch_helmholtz_t<cd>(b, kappa, kappa_im, f_grid, f_gamma, g_gamma, u_out, phi_inout, opts, stats,
                                     active);
    return batch_helmholtz_t<double>(b, kappa, kappa_im, f_grid, f_gamma, g_gamma, u_out, phi_inout, opts, stats,
                                     active);
}

bool batch_complex(const kfbi_batch *b) { return b->cplx; }

}  // namespace kfbi
