// Coarse tail of a periodic V-cycle (Sec. III.C): every level with at most
// TAIL_CELLS cells, down to the coarsest, handled by one workgroup with all of
// those levels' arrays in LDS.  On these grids a separate launch per step costs
// more than the step itself; here the whole sub-cycle is one launch.
//
// The arithmetic is the multi-kernel V-cycle's, step for step:
//   * fused red-black sweep with snapshot semantics (red from the old state,
//     black from the red-updated one), in place: each colour is computed into
//     registers, then written after a barrier;
//   * residual d = L(phi) - f + cbar, 8-child averages of phi and d, then
//     cbar <- (sum f + sum Q) / N for the level's later sweeps;
//   * coarse rhs f^H = L^H(R phi) - R d and cbar^H = (sum f^H + sum Q^H) / N^H;
//   * coarsest level: cbar from the current sum of Q before every sweep;
//   * cell-centred trilinear prolongation of phi^H - R phi (periodic wrap).
// Reductions run in a fixed order, so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace vmg {

namespace {

constexpr int TAIL_NT = 512;
constexpr int TAIL_POOL = 3 * TAIL_CELLS + 4 * (TAIL_CELLS / 8 + TAIL_CELLS / 64 + TAIL_CELLS / 512 + 1);

__device__ __forceinline__ int tw(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

struct TLev {
    int n0, n1, n2, N;
    double h2, inv_h2, inv_h4;
    double *phi, *old, *f, *del;   // LDS, x fastest, unpadded
};

__device__ __forceinline__ void tail_decode(const TLev& L, int e, int& i, int& j, int& k) {
    i = e % L.n0;
    const int r = e / L.n0;
    j = r % L.n1;
    k = r / L.n1;
}

__device__ __forceinline__ int tail_idx(const TLev& L, int i, int j, int k) {
    return (tw(k, L.n2) * L.n1 + tw(j, L.n1)) * L.n0 + tw(i, L.n0);
}

// Wrapped x offsets, row offsets and plane offsets of a cell and its two
// neighbours along each axis ([0] = -1, [1] = the cell, [2] = +1): every
// neighbour index is then a sum of three of them.
struct TNbr {
    int x[3], y[3], z[3];
};

__device__ __forceinline__ TNbr tail_nbr(int n0, int n1, int n2, int i, int j, int k) {
    TNbr o;
    const int p = n0 * n1;
    o.x[0] = i == 0 ? n0 - 1 : i - 1;
    o.x[1] = i;
    o.x[2] = i == n0 - 1 ? 0 : i + 1;
    o.y[0] = (j == 0 ? n1 - 1 : j - 1) * n0;
    o.y[1] = j * n0;
    o.y[2] = (j == n1 - 1 ? 0 : j + 1) * n0;
    o.z[0] = (k == 0 ? n2 - 1 : k - 1) * p;
    o.z[1] = k * p;
    o.z[2] = (k == n2 - 1 ? 0 : k + 1) * p;
    return o;
}

template <typename T>
__device__ __forceinline__ void tail_gather_o(const TNbr& o, const T* u, NbT<T>& v) {
    auto at = [&](int a, int b, int c) { return u[o.z[c] + o.y[b] + o.x[a]]; };
    v.xm = at(0, 1, 1);   v.xp = at(2, 1, 1);
    v.ym = at(1, 0, 1);   v.yp = at(1, 2, 1);
    v.zm = at(1, 1, 0);   v.zp = at(1, 1, 2);
    v.xpyp = at(2, 2, 1); v.xmym = at(0, 0, 1); v.xpym = at(2, 0, 1); v.xmyp = at(0, 2, 1);
    v.xpzp = at(2, 1, 2); v.xmzm = at(0, 1, 0); v.xpzm = at(2, 1, 0); v.xmzp = at(0, 1, 2);
    v.ypzp = at(1, 2, 2); v.ymzm = at(1, 0, 0); v.ypzm = at(1, 2, 0); v.ymzp = at(1, 0, 2);
}

template <typename T>
__device__ __forceinline__ void tail_gather(const TLev& L, const T* u, int i, int j, int k, NbT<T>& v) {
    tail_gather_o(tail_nbr(L.n0, L.n1, L.n2, i, j, k), u, v);
}

// Cell q of colour `colour` ((i+j+k) & 1) on an n0 x n1 x n2 grid with n0 even:
// q runs over the row-pairs' halves, so every thread works on a cell of the colour.
__device__ __forceinline__ void colour_cell(int n0, int n1, int q, int colour, int& i, int& j, int& k) {
    const int h = n0 >> 1;
    const int r = q / h;
    j = r % n1;
    k = r / n1;
    i = 2 * (q - r * h) + ((j + k + colour) & 1);
}

// Block-wide sums of two values in a fixed order; every thread gets the totals.
__device__ __forceinline__ void tail_sum2(double a, double b, double& A, double& B, double (*red)[2]) {
    a = wave_sum(a);
    b = wave_sum(b);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[w][0] = a;
        red[w][1] = b;
    }
    __syncthreads();
    A = 0.0;
    B = 0.0;
    for (int q = 0; q < TAIL_NT / 64; ++q) {
        A += red[q][0];
        B += red[q][1];
    }
    __syncthreads();
}

// One red-black sweep of level L: each colour's new values go to the LDS
// scratch plane tmp first and are copied into phi after a barrier, so every
// cell of a colour is computed from the same state.
__device__ void tail_sweep(const TLev& L, double* tmp, const Coef& c, double cb) {
    const int tid = threadIdx.x;
    auto update = [&](int i, int j, int k) {
        const int e = (k * L.n1 + j) * L.n0 + i;
        Nb v;
        tail_gather(L, L.phi, i, j, k, v);
        double S, D;
        const double Q = nl_root_d(v, L.del[e], c, L.inv_h4, S, D);
        tmp[e] = kink_relax(L.phi[e], (S - L.h2 * (Q + L.f[e] - cb)) * (1.0 / 6.0), D, kink_k(L.h2));
    };
    for (int colour = 0; colour < 2; ++colour) {
        if ((L.n0 & 1) == 0) {
            for (int q = tid; q < (L.N >> 1); q += TAIL_NT) {
                int i, j, k;
                colour_cell(L.n0, L.n1, q, colour, i, j, k);
                update(i, j, k);
            }
            __syncthreads();
            for (int q = tid; q < (L.N >> 1); q += TAIL_NT) {
                int i, j, k;
                colour_cell(L.n0, L.n1, q, colour, i, j, k);
                const int e = (k * L.n1 + j) * L.n0 + i;
                L.phi[e] = tmp[e];
            }
        } else {
            for (int e = tid; e < L.N; e += TAIL_NT) {
                int i, j, k;
                tail_decode(L, e, i, j, k);
                if (((i + j + k) & 1) == colour) update(i, j, k);
            }
            __syncthreads();
            for (int e = tid; e < L.N; e += TAIL_NT) {
                int i, j, k;
                tail_decode(L, e, i, j, k);
                if (((i + j + k) & 1) == colour) L.phi[e] = tmp[e];
            }
        }
        __syncthreads();
    }
}

// Descriptor of tail level l: sizes from the arguments, arrays carved out of
// the LDS pool in level order (phi, f, delta, and phiold below the top).  Built
// on the fly so that nothing is indexed by a run-time level in private memory.
__device__ __forceinline__ TLev tail_level(const TailArgs& a, double* pool, int l) {
    int off = 0;
    for (int q = 0; q < l; ++q) off += (q == 0 ? 3 : 4) * a.n[q][0] * a.n[q][1] * a.n[q][2];
    TLev T;
    T.n0 = a.n[l][0];
    T.n1 = a.n[l][1];
    T.n2 = a.n[l][2];
    T.N = T.n0 * T.n1 * T.n2;
    T.h2 = a.h[l] * a.h[l];
    T.inv_h2 = 1.0 / T.h2;
    T.inv_h4 = T.inv_h2 * T.inv_h2;
    T.phi = pool + off;
    T.f = T.phi + T.N;
    T.del = T.f + T.N;
    T.old = l > 0 ? T.del + T.N : nullptr;
    return T;
}

}  // namespace

__global__ void __launch_bounds__(TAIL_NT) k_tail(TailArgs a) {
    __shared__ double pool[TAIL_POOL];
    __shared__ double tmp[TAIL_CELLS];
    __shared__ double red[TAIL_NT / 64][2];
    __shared__ double cbar[TAIL_LEVELS];
    const int tid = threadIdx.x;
    const int nl = a.nlev;
    {
        const TLev T = tail_level(a, pool, 0);
        for (int e = tid; e < T.N; e += TAIL_NT) {
            T.phi[e] = a.phi[e];
            T.f[e] = a.f ? a.f[e] : 0.0;
        }
    }
    for (int l = 0; l < nl; ++l) {
        const TLev T = tail_level(a, pool, l);
        for (int e = tid; e < T.N; e += TAIL_NT) T.del[e] = a.delta[l][e];
    }
    if (tid == 0) cbar[0] = a.sc->cbar;
    __syncthreads();
    const int last = nl - 1;
    // ---- descent ------------------------------------------------------------
    for (int l = 0; l < last; ++l) {
        const TLev F = tail_level(a, pool, l);
        const TLev C = tail_level(a, pool, l + 1);
        for (int s = 0; s < a.nu1; ++s) tail_sweep(F, tmp, a.c, cbar[l]);
        // residual of every fine cell into tmp, then the 8-child averages of phi
        // and d (R d is kept as -R d in f^H); children are summed in a fixed order
        double sq = 0.0, sf = 0.0;
        for (int fe = tid; fe < F.N; fe += TAIL_NT) {
            int i, j, k;
            tail_decode(F, fe, i, j, k);
            Nb v;
            tail_gather(F, F.phi, i, j, k, v);
            double S;
            bool gd;
            const double Q = nl_root(v, F.del[fe], a.c, F.inv_h4, S, gd);
            tmp[fe] = (S - 6.0 * F.phi[fe]) * F.inv_h2 - Q - F.f[fe] + cbar[l];
            sq += Q;
            sf += F.f[fe];
        }
        __syncthreads();
        for (int e = tid; e < C.N; e += TAIL_NT) {
            int I, J, K;
            tail_decode(C, e, I, J, K);
            double sp = 0.0, sd = 0.0;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const int fe = ((2 * K + (m >> 2)) * F.n1 + 2 * J + ((m >> 1) & 1)) * F.n0 + 2 * I + (m & 1);
                sd += tmp[fe];
                sp += F.phi[fe];
            }
            C.phi[e] = 0.125 * sp;
            C.old[e] = 0.125 * sp;
            C.f[e] = -0.125 * sd;
        }
        double SQ, SF;
        tail_sum2(sq, sf, SQ, SF, red);   // also orders the restriction before the rhs
        if (tid == 0) cbar[l] = (SF + SQ) / (double)F.N;
        // coarse rhs f^H = L^H(R phi) - R d
        sq = 0.0;
        sf = 0.0;
        for (int e = tid; e < C.N; e += TAIL_NT) {
            int I, J, K;
            tail_decode(C, e, I, J, K);
            Nb v;
            tail_gather(C, C.phi, I, J, K, v);
            double S;
            bool gd;
            const double Q = nl_root(v, C.del[e], a.c, C.inv_h4, S, gd);
            const double fh = (S - 6.0 * C.phi[e]) * C.inv_h2 - Q + C.f[e];
            C.f[e] = fh;
            sq += Q;
            sf += fh;
        }
        tail_sum2(sq, sf, SQ, SF, red);
        if (tid == 0) cbar[l + 1] = (SF + SQ) / (double)C.N;
        __syncthreads();
    }
    // ---- coarsest level: cbar from the current sum of Q before every sweep ---
    {
        const TLev C = tail_level(a, pool, last);
        double sf = 0.0, dummy = 0.0, SF, D;
        for (int e = tid; e < C.N; e += TAIL_NT) sf += C.f[e];
        tail_sum2(sf, dummy, SF, D, red);
        for (int s = 0; s < a.ncoarse; ++s) {
            double sq = 0.0, SQ;
            for (int e = tid; e < C.N; e += TAIL_NT) {
                int i, j, k;
                tail_decode(C, e, i, j, k);
                Nb v;
                tail_gather(C, C.phi, i, j, k, v);
                double S;
                bool gd;
                sq += nl_root(v, C.del[e], a.c, C.inv_h4, S, gd);
            }
            tail_sum2(sq, dummy, SQ, D, red);
            tail_sweep(C, tmp, a.c, (SF + SQ) / (double)C.N);
        }
    }
    // ---- ascent: prolongation of the correction, post-smoothing -------------
    for (int l = last - 1; l >= 0; --l) {
        const TLev F = tail_level(a, pool, l);
        const TLev C = tail_level(a, pool, l + 1);
        for (int e = tid; e < F.N; e += TAIL_NT) {
            int i, j, k;
            tail_decode(F, e, i, j, k);
            const int I = i >> 1, J = j >> 1, K = k >> 1;
            const int si = (i & 1) ? 1 : -1, sj = (j & 1) ? 1 : -1, sk = (k & 1) ? 1 : -1;
            double acc = 0.0;
            for (int m = 0; m < 8; ++m) {
                const int ai = m & 1, aj = (m >> 1) & 1, ak = m >> 2;
                const double w = (ai ? 0.25 : 0.75) * (aj ? 0.25 : 0.75) * (ak ? 0.25 : 0.75);
                const int ci = tail_idx(C, I + ai * si, J + aj * sj, K + ak * sk);
                acc += w * (C.phi[ci] - C.old[ci]);
            }
            F.phi[e] += acc;
        }
        __syncthreads();
        for (int s = 0; s < a.nu2; ++s) tail_sweep(F, tmp, a.c, cbar[l]);
    }
    {
        const TLev T = tail_level(a, pool, 0);
        for (int e = tid; e < T.N; e += TAIL_NT) a.phi[e] = T.phi[e];
    }
    if (tid == 0) a.sc->cbar = cbar[0];
}

// ---------------------------------------------------------------------------
// Coarse tail of the mixed path's FP32 inner cycle: the same structure for the
// correction problem  Lap e - dQ(e) = r - cbar_e  (e, r, phi~, t0 per level).
// Below the tail's top level the base state phi~ is the 8-child average and
// t0 = +-sqrt|D0| comes from the FP64 discriminant of phi~ and delta, as in the
// multi-kernel inner cycle.
// ---------------------------------------------------------------------------
namespace {

constexpr int CTAIL_POOL = 4 * TAIL_CELLS + 5 * (TAIL_CELLS / 8 + TAIL_CELLS / 64 + TAIL_CELLS / 512 + 1);

struct CLev {
    int n0, n1, n2, N;
    float h2, inv_h2, a_ih4;
    double inv_h4;
    float *e, *r, *pt, *t0, *old;   // LDS
};

__device__ __forceinline__ CLev ctail_level(const TailCorrArgs& a, float* pool, int l) {
    int off = 0;
    for (int q = 0; q < l; ++q) off += (q == 0 ? 4 : 5) * a.n[q][0] * a.n[q][1] * a.n[q][2];
    CLev T;
    T.n0 = a.n[l][0];
    T.n1 = a.n[l][1];
    T.n2 = a.n[l][2];
    T.N = T.n0 * T.n1 * T.n2;
    const double h2 = a.h[l] * a.h[l];
    T.h2 = (float)h2;
    T.inv_h2 = (float)(1.0 / h2);
    T.inv_h4 = 1.0 / (h2 * h2);
    T.a_ih4 = (float)(a.c64.alpha * T.inv_h4);
    T.e = pool + off;
    T.r = T.e + T.N;
    T.pt = T.r + T.N;
    T.t0 = T.pt + T.N;
    T.old = l > 0 ? T.t0 + T.N : nullptr;
    return T;
}

__device__ __forceinline__ int ctail_idx(const CLev& L, int i, int j, int k) {
    return (tw(k, L.n2) * L.n1 + tw(j, L.n1)) * L.n0 + tw(i, L.n0);
}

__device__ __forceinline__ void ctail_decode(const CLev& L, int e, int& i, int& j, int& k) {
    i = e % L.n0;
    const int r = e / L.n0;
    j = r % L.n1;
    k = r / L.n1;
}

template <typename T>
__device__ __forceinline__ void ctail_gather(const CLev& L, const T* u, int i, int j, int k, NbT<T>& v) {
    tail_gather_o(tail_nbr(L.n0, L.n1, L.n2, i, j, k), u, v);
}

// dQ(e) at cell (i,j,k) and the neighbour sum of e
__device__ __forceinline__ float ctail_dq(const CLev& L, const CoefF& c, int i, int j, int k, int e, float& Se) {
    const TNbr o = tail_nbr(L.n0, L.n1, L.n2, i, j, k);
    NbT<float> ve, vp;
    tail_gather_o(o, L.e, ve);
    tail_gather_o(o, L.pt, vp);
    return dQ_of(dq_corr(ve, vp, L.a_ih4, Se), L.t0[e], c);
}

// ctail_dq that also returns the discriminant of the corrected state
__device__ __forceinline__ float ctail_dq_d(const CLev& L, const CoefF& c, int i, int j, int k, int e, float& Se,
                                            float& D1) {
    const TNbr o = tail_nbr(L.n0, L.n1, L.n2, i, j, k);
    NbT<float> ve, vp;
    tail_gather_o(o, L.e, ve);
    tail_gather_o(o, L.pt, vp);
    return dQ_of_d(dq_corr(ve, vp, L.a_ih4, Se), L.t0[e], c, D1);
}

__device__ void ctail_sweep(const CLev& L, float* tmp, const CoefF& c, float cb) {
    const int tid = threadIdx.x;
    auto update = [&](int i, int j, int k) {
        const int e = (k * L.n1 + j) * L.n0 + i;
        float Se, D1;
        const float dQ = ctail_dq_d(L, c, i, j, k, e, Se, D1);
        tmp[e] = kink_relax(L.e[e], (Se - L.h2 * (dQ + L.r[e] - cb)) * (1.0f / 6.0f), D1, kink_k(L.h2));
    };
    for (int colour = 0; colour < 2; ++colour) {
        if ((L.n0 & 1) == 0) {
            for (int q = tid; q < (L.N >> 1); q += TAIL_NT) {
                int i, j, k;
                colour_cell(L.n0, L.n1, q, colour, i, j, k);
                update(i, j, k);
            }
            __syncthreads();
            for (int q = tid; q < (L.N >> 1); q += TAIL_NT) {
                int i, j, k;
                colour_cell(L.n0, L.n1, q, colour, i, j, k);
                const int e = (k * L.n1 + j) * L.n0 + i;
                L.e[e] = tmp[e];
            }
        } else {
            for (int e = tid; e < L.N; e += TAIL_NT) {
                int i, j, k;
                ctail_decode(L, e, i, j, k);
                if (((i + j + k) & 1) == colour) update(i, j, k);
            }
            __syncthreads();
            for (int e = tid; e < L.N; e += TAIL_NT) {
                int i, j, k;
                ctail_decode(L, e, i, j, k);
                if (((i + j + k) & 1) == colour) L.e[e] = tmp[e];
            }
        }
        __syncthreads();
    }
}

}  // namespace

__global__ void __launch_bounds__(TAIL_NT) k_tail_corr(TailCorrArgs a) {
    __shared__ float pool[CTAIL_POOL];
    __shared__ float tmp[TAIL_CELLS];
    __shared__ double red[TAIL_NT / 64][2];
    __shared__ float cbar[TAIL_LEVELS];
    const int tid = threadIdx.x;
    const int nl = a.nlev;
    CoefF cf;
    cf.alpha = (float)a.c64.alpha;
    cf.c8 = (float)a.c64.c8;
    cf.a34 = a.c64.alpha != 0.0 ? (float)(3.0 / (4.0 * a.c64.alpha)) : 0.0f;
    {
        const CLev T = ctail_level(a, pool, 0);
        for (int e = tid; e < T.N; e += TAIL_NT) {
            T.e[e] = a.e[e];
            T.r[e] = a.r[e];
            T.pt[e] = a.pt[e];
            T.t0[e] = a.t0[e];
        }
    }
    if (tid == 0) cbar[0] = (float)a.sc->cbar;
    __syncthreads();
    const int last = nl - 1;
    for (int l = 0; l < last; ++l) {
        const CLev F = ctail_level(a, pool, l);
        const CLev C = ctail_level(a, pool, l + 1);
        for (int s = 0; s < a.nu1; ++s) ctail_sweep(F, tmp, cf, cbar[l]);
        // residual d_e of every fine cell into tmp, then the 8-child averages of
        // e, d_e (kept as -R d_e in r^H) and phi~, children summed in a fixed order
        double sq = 0.0, sf = 0.0;
        for (int fe = tid; fe < F.N; fe += TAIL_NT) {
            int i, j, k;
            ctail_decode(F, fe, i, j, k);
            float Se;
            const float dQ = ctail_dq(F, cf, i, j, k, fe, Se);
            tmp[fe] = (Se - 6.0f * F.e[fe]) * F.inv_h2 - dQ - F.r[fe] + cbar[l];
            sq += dQ;
            sf += F.r[fe];
        }
        __syncthreads();
        for (int e = tid; e < C.N; e += TAIL_NT) {
            int I, J, K;
            ctail_decode(C, e, I, J, K);
            float se = 0.0f, sd = 0.0f, sp = 0.0f;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const int fe = ((2 * K + (m >> 2)) * F.n1 + 2 * J + ((m >> 1) & 1)) * F.n0 + 2 * I + (m & 1);
                sd += tmp[fe];
                se += F.e[fe];
                sp += F.pt[fe];
            }
            C.e[e] = 0.125f * se;
            C.old[e] = 0.125f * se;
            C.r[e] = -0.125f * sd;
            C.pt[e] = 0.125f * sp;
        }
        double SQ, SF;
        tail_sum2(sq, sf, SQ, SF, red);
        if (tid == 0) cbar[l] = (float)((SF + SQ) / (double)F.N);
        // t0 of the coarse level from the FP64 discriminant of phi~ and delta
        for (int e = tid; e < C.N; e += TAIL_NT) {
            int I, J, K;
            ctail_decode(C, e, I, J, K);
            NbT<float> vp;
            ctail_gather(C, C.pt, I, J, K, vp);
            Nb vb;
            vb.xm = vp.xm; vb.xp = vp.xp; vb.ym = vp.ym; vb.yp = vp.yp; vb.zm = vp.zm; vb.zp = vp.zp;
            vb.xpyp = vp.xpyp; vb.xmym = vp.xmym; vb.xpym = vp.xpym; vb.xmyp = vp.xmyp;
            vb.xpzp = vp.xpzp; vb.xmzm = vp.xmzm; vb.xpzm = vp.xpzm; vb.xmzp = vp.xmzp;
            vb.ypzp = vp.ypzp; vb.ymzm = vp.ymzm; vb.ypzm = vp.ypzm; vb.ymzp = vp.ymzp;
            const double D0 = base_discriminant(vb, a.delta[l + 1][e], a.c64, C.inv_h4);
            C.t0[e] = (float)(D0 >= 0.0 ? sqrt(D0) : -sqrt(-D0));
        }
        __syncthreads();
        // coarse rhs r^H = L_e^H(R e) - R d_e
        sq = 0.0;
        sf = 0.0;
        for (int e = tid; e < C.N; e += TAIL_NT) {
            int I, J, K;
            ctail_decode(C, e, I, J, K);
            float Se;
            const float dQ = ctail_dq(C, cf, I, J, K, e, Se);
            const float rh = (Se - 6.0f * C.e[e]) * C.inv_h2 - dQ + C.r[e];
            C.r[e] = rh;
            sq += dQ;
            sf += rh;
        }
        tail_sum2(sq, sf, SQ, SF, red);
        if (tid == 0) cbar[l + 1] = (float)((SF + SQ) / (double)C.N);
        __syncthreads();
    }
    // coarsest level: cbar_e from the current sum of dQ before every sweep
    {
        const CLev C = ctail_level(a, pool, last);
        double sf = 0.0, dummy = 0.0, SF, D;
        for (int e = tid; e < C.N; e += TAIL_NT) sf += C.r[e];
        tail_sum2(sf, dummy, SF, D, red);
        for (int s = 0; s < a.ncoarse; ++s) {
            double sq = 0.0, SQ;
            for (int e = tid; e < C.N; e += TAIL_NT) {
                int i, j, k;
                ctail_decode(C, e, i, j, k);
                float Se;
                sq += ctail_dq(C, cf, i, j, k, e, Se);
            }
            tail_sum2(sq, dummy, SQ, D, red);
            ctail_sweep(C, tmp, cf, (float)((SF + SQ) / (double)C.N));
        }
    }
    // ascent: prolongation of the correction's correction, post-smoothing
    for (int l = last - 1; l >= 0; --l) {
        const CLev F = ctail_level(a, pool, l);
        const CLev C = ctail_level(a, pool, l + 1);
        for (int e = tid; e < F.N; e += TAIL_NT) {
            int i, j, k;
            ctail_decode(F, e, i, j, k);
            const int I = i >> 1, J = j >> 1, K = k >> 1;
            const int si = (i & 1) ? 1 : -1, sj = (j & 1) ? 1 : -1, sk = (k & 1) ? 1 : -1;
            float acc = 0.0f;
            for (int m = 0; m < 8; ++m) {
                const int ai = m & 1, aj = (m >> 1) & 1, ak = m >> 2;
                const float w = (ai ? 0.25f : 0.75f) * (aj ? 0.25f : 0.75f) * (ak ? 0.25f : 0.75f);
                const int ci = ctail_idx(C, I + ai * si, J + aj * sj, K + ak * sk);
                acc += w * (C.e[ci] - C.old[ci]);
            }
            F.e[e] += acc;
        }
        __syncthreads();
        for (int s = 0; s < a.nu2; ++s) ctail_sweep(F, tmp, cf, cbar[l]);
    }
    {
        const CLev T = ctail_level(a, pool, 0);
        for (int e = tid; e < T.N; e += TAIL_NT) a.e[e] = T.e[e];
    }
    if (tid == 0) a.sc->cbar = cbar[0];
}

hipError_t launch_tail_corr(const TailCorrArgs& a, hipStream_t s) {
    if (a.nlev < 1 || a.nlev > TAIL_LEVELS) return hipErrorInvalidValue;
    int64_t need = 0;
    for (int l = 0; l < a.nlev; ++l) {
        const int64_t N = (int64_t)a.n[l][0] * a.n[l][1] * a.n[l][2];
        if (N > TAIL_CELLS || a.n[l][0] < 1 || a.n[l][1] < 1 || a.n[l][2] < 1) return hipErrorInvalidValue;
        if (l > 0)
            for (int d = 0; d < 3; ++d)
                if (2 * a.n[l][d] != a.n[l - 1][d]) return hipErrorInvalidValue;
        need += (l == 0 ? 4 : 5) * N;
    }
    if (need > CTAIL_POOL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_tail_corr, dim3(1), dim3(TAIL_NT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_tail(const TailArgs& a, hipStream_t s) {
    if (a.nlev < 1 || a.nlev > TAIL_LEVELS) return hipErrorInvalidValue;
    int64_t need = 0;
    for (int l = 0; l < a.nlev; ++l) {
        const int64_t N = (int64_t)a.n[l][0] * a.n[l][1] * a.n[l][2];
        if (N > TAIL_CELLS || a.n[l][0] < 1 || a.n[l][1] < 1 || a.n[l][2] < 1) return hipErrorInvalidValue;
        if (l > 0)
            for (int d = 0; d < 3; ++d)
                if (2 * a.n[l][d] != a.n[l - 1][d]) return hipErrorInvalidValue;
        need += (l == 0 ? 3 : 4) * N;
    }
    if (need > TAIL_POOL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_tail, dim3(1), dim3(TAIL_NT), 0, s, a);
    return hipGetLastError();
}

}  // namespace vmg
