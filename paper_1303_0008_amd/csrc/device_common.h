// Device helpers shared by the FP64 and mixed-precision kernel files.
#pragma once
#include "vmg_internal.h"

namespace vmg {

constexpr int NT = 256;          // threads per block for every kernel here
constexpr int MAX_RED_BLOCKS = 2048;

__device__ __forceinline__ int wrapi(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}


// ---------------------------------------------------------------------------
// Raw buffer access (gfx9 buffer resource).  A load whose byte offset is at or
// beyond the resource's record count returns 0 and such a store is dropped, so
// tile edges and masked cells need no branch around the memory instruction:
// every lane issues every load and store, and the compiler can count the
// outstanding memory operations exactly (a branch around a load makes it wait
// for all of them, which would stall a software pipeline on its own
// prefetches).  A resource covers one z plane of an array: its base is the
// plane's first element and in-plane offsets stay 32-bit.
// ---------------------------------------------------------------------------
constexpr int BUF_RECORDS = 0x7FFFFFF0;    // bytes a plane resource covers
constexpr int BUF_OOB = 0x7FFFFFF8;        // byte offset of a masked access (out of range)
constexpr int BUF_WORD3 = 0x00020000;      // gfx9 resource word 3: 32-bit data format, raw access

// resource for the array element at index `elem` (may be negative: the
// plane's in-plane offsets bring the address back into the array) of an array
// of `eb`-byte elements; `ok` false makes every access through it out of range
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* base, int64_t elem, int eb, bool ok) {
    const uintptr_t a = reinterpret_cast<uintptr_t>(base) + (uintptr_t)(elem * eb);
    return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(a), (short)0, ok ? BUF_RECORDS : 0, BUF_WORD3);
}

typedef unsigned int vmg_u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double buf_ld_f64(__amdgpu_buffer_rsrc_t r, int bo) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, bo, 0, 0));
}
__device__ __forceinline__ float buf_ld_f32(__amdgpu_buffer_rsrc_t r, int bo) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, bo, 0, 0));
}
__device__ __forceinline__ void buf_st_f64(__amdgpu_buffer_rsrc_t r, int bo, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(vmg_u32x2, v), r, bo, 0, 0);
}
__device__ __forceinline__ void buf_st_f32(__amdgpu_buffer_rsrc_t r, int bo, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, bo, 0, 0);
}

// 18 stencil neighbours of a cell (the centre is not needed by the root).
template <typename T>
struct NbT {
    T xm, xp, ym, yp, zm, zp;
    T xpyp, xmym, xpym, xmyp;
    T xpzp, xmzm, xpzm, xmzp;
    T ypzp, ymzm, ypzm, ymzp;
};
using Nb = NbT<double>;

// Reciprocal and square root from the hardware approximations (v_rcp_f64,
// v_rsq_f64) refined by two Newton steps each: ~1 ulp, a third of the IEEE
// division / square-root sequences.
__device__ __forceinline__ double rcp_nr(double u) {
    double r = __builtin_amdgcn_rcp(u);
    double e = fma(-u, r, 1.0);
    r = fma(r, e, r);
    e = fma(-u, r, 1.0);
    return fma(r, e, r);
}

__device__ __forceinline__ double sqrt_nr(double D) {   // D > 0
    const double y = __builtin_amdgcn_rsq(D);
    const double hy = 0.5 * y;
    double s = D * y;
    s = fma(hy, fma(-s, s, D), s);
    return fma(hy, fma(-s, s, D), s);
}

// Right-hand side q = alpha Sigma0 + kappa delta of a cell's quadratic (Sec. III.A)
// from its 18 neighbours (Sigma0 h^4 = (dxy^2 + dxz^2 + dyz^2)/3 + (bxy^2 + bxz^2 +
// byz^2)/8, the phi_c-free part of (Lap phi)^2 - (d_i d_j phi)^2 at w = 1/3); also
// the neighbour sum S.  alpha/h^4 is folded into the two weights, which are
// kernel constants.
__device__ __forceinline__ double nl_q(const Nb& v, double dl, const Coef& c, double inv_h4, double& S) {
    const double sx = v.xp + v.xm, sy = v.yp + v.ym, sz = v.zp + v.zm;
    S = sx + sy + sz;
    const double dxy = sx - sy, dxz = sx - sz, dyz = sy - sz;
    const double bxy = (v.xpyp + v.xmym) - (v.xpym + v.xmyp);
    const double bxz = (v.xpzp + v.xmzm) - (v.xpzm + v.xmzp);
    const double byz = (v.ypzp + v.ymzm) - (v.ypzm + v.ymzp);
    const double sd = fma(dxy, dxy, fma(dxz, dxz, dyz * dyz));
    const double sb = fma(bxy, bxy, fma(bxz, bxz, byz * byz));
    const double a3 = c.alpha * inv_h4 * (1.0 / 3.0), a8 = c.alpha * inv_h4 * 0.125;
    return fma(a3, sd, fma(a8, sb, c.kappa * dl));
}

// Physical root Q of the per-cell quadratic (Sec. III.A, Eq. one_branch at w = 1/3)
// from D = 1 + 8 alpha q / 3 > 0: Q = 2q / (1 + sqrt D) = (sqrt D - 1) 3 / (4 alpha).
// The second form needs no division; its cancellation near D = 1 costs an
// absolute error of about eps sqrt(D) 3 / (4 |alpha|), below the rounding of
// the residual when |alpha| >= 1e-2 (Coef::sqrt_form), else the first is used.
__device__ __forceinline__ double nl_root_of(double q, double sD, const Coef& c) {
    return c.sqrt_form ? fma(sD, -c.vertex, c.vertex) : 2.0 * q * rcp_nr(1.0 + sD);
}

// Q and S of a cell and the guard flag (D <= 0: the vertex -3 / (4 alpha); D == 0
// gives the vertex from either form, so the guard branch is continuous there).
__device__ __forceinline__ double nl_root(const Nb& v, double dl, const Coef& c, double inv_h4,
                                          double& S, bool& guard) {
    const double q = nl_q(v, dl, c, inv_h4, S);
    const double D = fma(c.c8, q, 1.0);
    guard = !(D > 0.0);
    return guard ? c.vertex : nl_root_of(q, sqrt_nr(D), c);
}

// nl_root that also returns the discriminant D (the smoothers' kink test).
__device__ __forceinline__ double nl_root_d(const Nb& v, double dl, const Coef& c, double inv_h4,
                                            double& S, double& D) {
    const double q = nl_q(v, dl, c, inv_h4, S);
    D = fma(c.c8, q, 1.0);
    return !(D > 0.0) ? c.vertex : nl_root_of(q, sqrt_nr(D), c);
}

// Kink cells.  Near D = 0 the root's slope 1/sqrt(D) (Eq. one_branch) couples
// a cell so strongly to its neighbours that the plain Gauss-Seidel update can
// oscillate across D = 0 from one sweep to the next (clamped on one sweep, on
// the steep side of the root on the next) and the solve stalls.  The coupling
// grows like 1 / (h^2 sqrt|D|) (the root's slope times the neighbours' weight
// in q, alpha / h^4, times the update's h^2 / 6), so the update is
// under-relaxed by w = min(1, max(KINK_WMIN, KINK_K h^2 sqrt|D|)); w = 1 (the
// update itself, bit for bit) wherever KINK_K h^2 sqrt|D| >= 1.  A converged
// state is a fixed point either way, so the discrete solution is unchanged.
// Every smoother (both precisions, every schedule) applies the same rule, so
// schedules stay bitwise interchangeable.  kink_k(h^2) is the per-level factor
// KINK_K h^2.
constexpr double KINK_K = 50.0 * 65536.0;   // w = 50 sqrt|D| on a 256^3 unit box
constexpr float KINK_WMIN = 0.01f;

__host__ __device__ __forceinline__ float kink_k(double h2) { return (float)(KINK_K * h2); }

// (kk^2 |D| < 1 is tested first, so that a wave without kink cells, nearly
// every wave, branches past the weight)
__device__ __forceinline__ double kink_relax(double old, double nv, double D, float kk) {
    const float aD = (float)fabs(D);
    if (__builtin_expect(aD * (kk * kk) < 1.0f, 0)) {
        const float w = fmaxf(kk * __builtin_amdgcn_sqrtf(aD), KINK_WMIN);
        return fma((double)fminf(w, 1.0f), nv - old, old);
    }
    return nv;
}

// kink_relax with the old value read from LDS inside the rare branch
__device__ __forceinline__ double kink_relax_at(const double* pold, double nv, double D, float kk) {
    const float aD = (float)fabs(D);
    if (__builtin_expect(aD * (kk * kk) < 1.0f, 0)) {
        const double old = *(const volatile double*)pold;
        const float w = fmaxf(kk * __builtin_amdgcn_sqrtf(aD), KINK_WMIN);
        return fma((double)fminf(w, 1.0f), nv - old, old);
    }
    return nv;
}

__device__ __forceinline__ float kink_relax(float old, float nv, float D, float kk) {
    const float aD = fabsf(D);
    if (__builtin_expect(aD * (kk * kk) < 1.0f, 0)) {
        const float w = fmaxf(kk * __builtin_amdgcn_sqrtf(aD), KINK_WMIN);
        return fmaf(fminf(w, 1.0f), nv - old, old);
    }
    return nv;
}

// nl_root that also returns the discriminant D and +-sqrt|D| (sign of D): the
// outer FP64 pass of the mixed path hands +-sqrt|D0| to the FP32 inner problem.
__device__ __forceinline__ double nl_root_t0(const Nb& v, double dl, const Coef& c, double inv_h4,
                                             double& S, bool& guard, double& t0) {
    const double q = nl_q(v, dl, c, inv_h4, S);
    const double D = fma(c.c8, q, 1.0);
    guard = !(D > 0.0);
    if (guard) {
        t0 = D < 0.0 ? -sqrt_nr(-D) : 0.0;
        return c.vertex;
    }
    const double sD = sqrt_nr(D);
    t0 = sD;
    return nl_root_of(q, sD, c);
}

// Discriminant D = 1 + 8 alpha q / 3 of a cell's quadratic (Sec. III.A) from
// its 18 neighbours and density (the mixed path's base state).
__device__ __forceinline__ double base_discriminant(const Nb& v, double dl, const Coef& c, double inv_h4) {
    double S;
    return fma(c.c8, nl_q(v, dl, c, inv_h4, S), 1.0);
}

// Correction of the mixed path's FP32 inner problem: dq = alpha Phi(2 phi~ + e, e)
// / h^4 from the neighbourhoods of e and of the base state phi~ (Phi the
// bilinear form of Sigma0), and dQ = Q(q0 + dq) - Q(q0) from t0 = +-sqrt|D0|.
__device__ __forceinline__ float dq_corr(const NbT<float>& e, const NbT<float>& p, float a_ih4,
                                         float& Se) {
    const float sxe = e.xp + e.xm, sye = e.yp + e.ym, sze = e.zp + e.zm;
    const float sxp = p.xp + p.xm, syp = p.yp + p.ym, szp = p.zp + p.zm;
    Se = sxe + sye + sze;
    const float dxy_e = sxe - sye, dxz_e = sxe - sze, dyz_e = sye - sze;
    const float dxy_w = 2.0f * (sxp - syp) + dxy_e;
    const float dxz_w = 2.0f * (sxp - szp) + dxz_e;
    const float dyz_w = 2.0f * (syp - szp) + dyz_e;
    const float bxy_e = (e.xpyp + e.xmym) - (e.xpym + e.xmyp);
    const float bxz_e = (e.xpzp + e.xmzm) - (e.xpzm + e.xmzp);
    const float byz_e = (e.ypzp + e.ymzm) - (e.ypzm + e.ymzp);
    const float bxy_w = 2.0f * ((p.xpyp + p.xmym) - (p.xpym + p.xmyp)) + bxy_e;
    const float bxz_w = 2.0f * ((p.xpzp + p.xmzm) - (p.xpzm + p.xmzp)) + bxz_e;
    const float byz_w = 2.0f * ((p.ypzp + p.ymzm) - (p.ypzm + p.ymzp)) + byz_e;
    const float pd = fmaf(dxy_w, dxy_e, fmaf(dxz_w, dxz_e, dyz_w * dyz_e));
    const float pb = fmaf(bxy_w, bxy_e, fmaf(bxz_w, bxz_e, byz_w * byz_e));
    // alpha/h^4 folded into the weights 1/3 and 1/8 (kernel constants)
    return fmaf(a_ih4 * (1.0f / 3.0f), pd, a_ih4 * 0.125f * pb);
}

// dQ_of that also returns the discriminant D1 of the corrected state (the
// smoothers' kink test)
__device__ __forceinline__ float dQ_of_d(float dq, float t0, const CoefF& c, float& D1) {
    const float D0 = t0 * fabsf(t0);   // sign(t0) t0^2
    const float s0 = fmaxf(t0, 0.0f);
    D1 = fmaf(c.c8, dq, D0);
    const float s1 = __builtin_amdgcn_sqrtf(fmaxf(D1, 0.0f));
    if (D0 >= 0.0f && D1 >= 0.0f) {
        const float den = s0 + s1;
        return den > 0.0f ? 2.0f * dq * __builtin_amdgcn_rcpf(den) : 0.0f;
    }
    return c.a34 * (s1 - s0);
}

__device__ __forceinline__ float dQ_of(float dq, float t0, const CoefF& c) {
    const float D0 = t0 * fabsf(t0);   // sign(t0) t0^2
    const float s0 = fmaxf(t0, 0.0f);
    const float D1 = fmaf(c.c8, dq, D0);
    const float s1 = __builtin_amdgcn_sqrtf(fmaxf(D1, 0.0f));
    if (D0 >= 0.0f && D1 >= 0.0f) {
        const float den = s0 + s1;
        return den > 0.0f ? 2.0f * dq * __builtin_amdgcn_rcpf(den) : 0.0f;
    }
    return c.a34 * (s1 - s0);
}

// Column X of an LDS tile row of even width W stored split by parity (even
// columns first).  A lane handling cells X = 2m+1 and 2m+2 then reads each
// neighbour column from consecutive words across lanes (no bank conflicts).
template <int W>
__device__ __forceinline__ int split_col(int X) {
    static_assert(W % 2 == 0, "split rows need an even width");
    return (X & 1) * (W / 2) + (X >> 1);
}

__device__ __forceinline__ int xcd_remap(int b, int nb) {
    // Blocks are dispatched round-robin over the 8 XCDs; give each XCD a
    // contiguous range of tiles so that shared halos stay in one L2.
    if ((nb & 7) != 0) return b;
    return (b & 7) * (nb >> 3) + (b >> 3);
}

__device__ __forceinline__ void decode(const Geom& g, int64_t e, int& i, int& j, int& k) {
    if (g.ncell <= 0x7fffffff) {
        // 32-bit division: a few instructions against the long software
        // sequence of a 64-bit one (every grid below 2^31 cells)
        const unsigned u = (unsigned)e, n0 = (unsigned)g.n0, n1 = (unsigned)g.n1;
        const unsigned r = u / n0;
        i = (int)(u - r * n0);
        const unsigned kk = r / n1;
        j = (int)(r - kk * n1);
        k = (int)kk;
        return;
    }
    i = (int)(e % g.n0);
    const int64_t r = e / g.n0;
    j = (int)(r % g.n1);
    k = (int)(r / g.n1);
}

__device__ __forceinline__ int64_t cell_index(const Geom& g, int i, int j, int k) {
    return g.off0 + i + (int64_t)j * g.sy + (int64_t)k * g.sz;
}

// 18 neighbours of cell (i,j,k) read through global memory (periodic wrap or ghost shell)
template <int DIR, typename T, typename NB>
__device__ __forceinline__ T gather_nb(const Geom& g, const T* __restrict__ u, int i, int j, int k, NB& v) {
    int im, ip, jm, jp, km, kp;
    if (DIR) {
        im = i - 1; ip = i + 1; jm = j - 1; jp = j + 1; km = k - 1; kp = k + 1;
    } else {
        im = i == 0 ? g.n0 - 1 : i - 1; ip = i == g.n0 - 1 ? 0 : i + 1;
        jm = j == 0 ? g.n1 - 1 : j - 1; jp = j == g.n1 - 1 ? 0 : j + 1;
        km = k == 0 ? g.n2 - 1 : k - 1; kp = k == g.n2 - 1 ? 0 : k + 1;
    }
    const int64_t sy = g.sy, sz = g.sz, o = g.off0;
    auto at = [&](int x, int y, int z) { return u[o + x + y * sy + z * sz]; };
    v.xm = at(im, j, k); v.xp = at(ip, j, k);
    v.ym = at(i, jm, k); v.yp = at(i, jp, k);
    v.zm = at(i, j, km); v.zp = at(i, j, kp);
    v.xpyp = at(ip, jp, k); v.xmym = at(im, jm, k); v.xpym = at(ip, jm, k); v.xmyp = at(im, jp, k);
    v.xpzp = at(ip, j, kp); v.xmzm = at(im, j, km); v.xpzm = at(ip, j, km); v.xmzp = at(im, j, kp);
    v.ypzp = at(i, jp, kp); v.ymzm = at(i, jm, km); v.ypzm = at(i, jp, km); v.ymzp = at(i, jm, kp);
    return at(i, j, k);
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sum R_NSLOT per-thread accumulators over the block (fixed order) and store
// them in partials[blockIdx.x * R_NSLOT + k].
__device__ __forceinline__ void block_store_partials(double (&acc)[R_NSLOT], double* partials) {
    __shared__ double red[NT / 64][R_NSLOT];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < R_NSLOT; ++k) {
        const double s = wave_sum(acc[k]);
        if (lane == 0) red[w][k] = s;
    }
    __syncthreads();
    if (threadIdx.x < R_NSLOT) {
        double s = 0.0;
        for (int q = 0; q < NT / 64; ++q) s += red[q][threadIdx.x];
        partials[(int64_t)blockIdx.x * R_NSLOT + threadIdx.x] = s;
    }
}

// Per-item passes of the batched plans run one wave per item of ITEM_CELLS cells,
// each lane taking ITEM_CELLS / 64 of them, so that the cross-lane sums of the
// partials are paid once per item rather than once per 64 cells.
constexpr int ITEM_LANES = 64;
static_assert(ITEM_CELLS == NT, "the one-thread-per-cell item passes run NT threads per item");

// Sum R_NSLOT per-lane accumulators over a one-wave block and store them in
// partials[blockIdx.x * R_NSLOT + k].
__device__ __forceinline__ void wave_store_partials(double (&acc)[R_NSLOT], double* partials) {
#pragma unroll
    for (int k = 0; k < R_NSLOT; ++k) {
        const double s = wave_sum(acc[k]);
        if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * R_NSLOT + k] = s;
    }
}

// residual d = L(phi) + cbar - f at one cell; also returns Q and the guard flag
template <int DIR>
__device__ __forceinline__ double cell_residual(const Geom& g, const Coef& c, const double* phi,
                                                const double* delta, const double* f, double cb,
                                                int i, int j, int k, double inv_h2, double inv_h4,
                                                double& Q, bool& gd, double& pc, double& fv) {
    Nb v;
    pc = gather_nb<DIR>(g, phi, i, j, k, v);
    const int64_t gi = cell_index(g, i, j, k);
    double S;
    Q = nl_root(v, delta[gi], c, inv_h4, S, gd);
    fv = f ? f[gi] : 0.0;
    return (S - 6.0 * pc) * inv_h2 - Q - fv + cb;
}

// Mirror an index that lies one cell outside [0, n) back inside; each mirrored
// axis flips the sign of a correction (homogeneous Dirichlet data on the cell
// faces of a cell-centred grid).
__device__ __forceinline__ int mirror(int i, int n, int& sign) {
    if (i < 0) { sign = -sign; return 0; }
    if (i >= n) { sign = -sign; return n - 1; }
    return i;
}

// Trilinear prolongation of a Dirichlet grid's coarse correction uc - oc onto the
// 8 children (2I+a, 2J+b, 2K+c) of coarse cell (I, J, K), added to uf: the 3^3
// coarse neighbourhood is read once (mirrored, with a sign flip, one cell outside
// the grid) and each child sums its 8 nearest coarse values with weights 3/4 and
// 1/4 per axis, in the same order as a child taken on its own.
template <typename T>
__device__ __forceinline__ void prolong_children(const Geom& gf, const Geom& gc, T* __restrict__ uf,
                                                 const T* __restrict__ uc, const T* __restrict__ oc, int I, int J,
                                                 int K) {
    int ix[3], jy[3], kz[3], sx[3], sy[3], sz[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        sx[d] = sy[d] = sz[d] = 1;
        ix[d] = mirror(I + d - 1, gc.n0, sx[d]);
        jy[d] = mirror(J + d - 1, gc.n1, sy[d]);
        kz[d] = mirror(K + d - 1, gc.n2, sz[d]);
    }
    T dl[3][3][3];
#pragma unroll
    for (int z = 0; z < 3; ++z)
#pragma unroll
        for (int y = 0; y < 3; ++y) {
            const int64_t row = gc.off0 + (int64_t)jy[y] * gc.sy + (int64_t)kz[z] * gc.sz;
#pragma unroll
            for (int x = 0; x < 3; ++x) {
                const int64_t ci = row + ix[x];
                const T sgn = (T)(sx[x] * sy[y] * sz[z]);
                dl[z][y][x] = sgn * (uc[ci] - oc[ci]);
            }
        }
#pragma unroll
    for (int ch = 0; ch < 8; ++ch) {
        const int a = ch & 1, b = (ch >> 1) & 1, c = ch >> 2;
        T acc = (T)0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int x = 1 + ((q & 1) ? (a ? 1 : -1) : 0);
            const int y = 1 + ((q & 2) ? (b ? 1 : -1) : 0);
            const int z = 1 + ((q & 4) ? (c ? 1 : -1) : 0);
            const T wq = (T)(((q & 1) ? 0.25 : 0.75) * ((q & 2) ? 0.25 : 0.75) * ((q & 4) ? 0.25 : 0.75));
            acc += wq * dl[z][y][x];
        }
        uf[cell_index(gf, 2 * I + a, 2 * J + b, 2 * K + c)] += acc;
    }
}

// Right after a restriction, u = ref on every interior cell of a coarse
// Dirichlet level, so its refreshed ghost shell (ref + (-1)^k (u - ref) at the
// mirrored cell) is ref's.  The thread of interior cell (I, J, K) copies the
// face and edge ghosts whose mirrored cell it is: each ghost has one writer.
template <typename T>
__device__ __forceinline__ void copy_ghosts_near(const Geom& g, T* __restrict__ u, const T* __restrict__ ref, int I,
                                                 int J, int K) {
    if (I > 0 && I < g.n0 - 1 && J > 0 && J < g.n1 - 1 && K > 0 && K < g.n2 - 1) return;
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                const int out = (dx != 0) + (dy != 0) + (dz != 0);
                if (out == 0 || out == 3) continue;   // the cell itself; corners are not stored
                const int x = I + dx, y = J + dy, z = K + dz;
                if ((dx != 0 && x >= 0 && x < g.n0) || (dy != 0 && y >= 0 && y < g.n1) ||
                    (dz != 0 && z >= 0 && z < g.n2))
                    continue;                         // a step that stays inside: not a ghost of this cell
                const int64_t gi = cell_index(g, x, y, z);
                u[gi] = ref[gi];
            }
}

// The 4^3 block of a padded (Dirichlet) fine grid around the children of coarse
// cell (I, J, K), corners left out: b[z][y][x] = u at fine cell (2I-1+x, 2J-1+y,
// 2K-1+z).  The 18-point stencils of the 8 children read exactly these 56 values.
template <typename T>
__device__ __forceinline__ void load_child_box(const Geom& g, const T* __restrict__ u, int I, int J, int K,
                                               T (&b)[4][4][4]) {
    const int64_t o = cell_index(g, 2 * I - 1, 2 * J - 1, 2 * K - 1);
#pragma unroll
    for (int z = 0; z < 4; ++z)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
            const int64_t row = o + (int64_t)y * g.sy + (int64_t)z * g.sz;
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                const bool corner = (x == 0 || x == 3) && (y == 0 || y == 3) && (z == 0 || z == 3);
                b[z][y][x] = corner ? (T)0 : u[row + x];
            }
        }
}

// stencil of child (a, b, c) out of a child box; returns the centre value
template <typename T>
__device__ __forceinline__ T box_nb(const T (&u)[4][4][4], int a, int b, int c, NbT<T>& v) {
    const int x = 1 + a, y = 1 + b, z = 1 + c;
    v.xm = u[z][y][x - 1]; v.xp = u[z][y][x + 1];
    v.ym = u[z][y - 1][x]; v.yp = u[z][y + 1][x];
    v.zm = u[z - 1][y][x]; v.zp = u[z + 1][y][x];
    v.xpyp = u[z][y + 1][x + 1]; v.xmym = u[z][y - 1][x - 1]; v.xpym = u[z][y - 1][x + 1]; v.xmyp = u[z][y + 1][x - 1];
    v.xpzp = u[z + 1][y][x + 1]; v.xmzm = u[z - 1][y][x - 1]; v.xpzm = u[z - 1][y][x + 1]; v.xmzp = u[z + 1][y][x - 1];
    v.ypzp = u[z + 1][y + 1][x]; v.ymzm = u[z - 1][y - 1][x]; v.ypzm = u[z - 1][y + 1][x]; v.ymzp = u[z + 1][y - 1][x];
    return u[z][y][x];
}

__device__ __forceinline__ int64_t ghost_count_dev(int n0, int n1, int n2) {
    return 2 * ((int64_t)n1 * n2 + (int64_t)n0 * n2 + (int64_t)n0 * n1) + 4 * ((int64_t)n0 + n1 + n2);
}

// Decode a compact ghost index into cell coordinates (i, j, k) in [-1, n]
// (integer type I: 32-bit when the shell has fewer than 2^31 values).
template <typename I>
__device__ __forceinline__ void ghost_coords_t(I n0, I n1, I n2, I q, int& i, int& j, int& k) {
    const I fx = n1 * n2, fy = n0 * n2, fz = n0 * n1;
    if (q < 2 * fx) { const int s = (int)(q / fx); const I r = q - (I)s * fx;
        i = s ? (int)n0 : -1; j = (int)(r % n1); k = (int)(r / n1); return; }
    q -= 2 * fx;
    if (q < 2 * fy) { const int s = (int)(q / fy); const I r = q - (I)s * fy;
        j = s ? (int)n1 : -1; i = (int)(r % n0); k = (int)(r / n0); return; }
    q -= 2 * fy;
    if (q < 2 * fz) { const int s = (int)(q / fz); const I r = q - (I)s * fz;
        k = s ? (int)n2 : -1; i = (int)(r % n0); j = (int)(r / n0); return; }
    q -= 2 * fz;
    if (q < 4 * n0) { const int e = (int)(q / n0);
        i = (int)(q - (I)e * n0); j = (e & 1) ? (int)n1 : -1; k = (e & 2) ? (int)n2 : -1; return; }
    q -= 4 * n0;
    if (q < 4 * n1) { const int e = (int)(q / n1);
        j = (int)(q - (I)e * n1); i = (e & 1) ? (int)n0 : -1; k = (e & 2) ? (int)n2 : -1; return; }
    q -= 4 * n1;
    const int e = (int)(q / n2);
    k = (int)(q - (I)e * n2); i = (e & 1) ? (int)n0 : -1; j = (e & 2) ? (int)n1 : -1;
}

__device__ __forceinline__ void ghost_coords(int n0, int n1, int n2, int64_t q, int& i, int& j, int& k) {
    if (ghost_count_dev(n0, n1, n2) <= 0x7fffffff)
        ghost_coords_t<unsigned>((unsigned)n0, (unsigned)n1, (unsigned)n2, (unsigned)q, i, j, k);
    else
        ghost_coords_t<int64_t>(n0, n1, n2, q, i, j, k);
}

// Coarse Dirichlet ghost refresh: ghost = reference + (-1)^k (u - ref) at the mirrored
// interior cell, i.e. the coarse correction u - ref vanishes on the grid faces.
template <typename T>
__global__ void k_ghost_refresh_batch(const Geom* __restrict__ gs, const int2* __restrict__ items, T* u,
                                      const T* __restrict__ ref) {
    const int2 w = items[blockIdx.x];
    const Geom g = gs[w.x];
    const int64_t q = (int64_t)w.y + threadIdx.x;
    if (q >= ghost_count_dev(g.n0, g.n1, g.n2)) return;
    int i, j, k;
    ghost_coords(g.n0, g.n1, g.n2, q, i, j, k);
    int sign = 1;
    const int ir = mirror(i, g.n0, sign), jr = mirror(j, g.n1, sign), kr = mirror(k, g.n2, sign);
    const int64_t gi = cell_index(g, i, j, k), ii = cell_index(g, ir, jr, kr);
    u[gi] = ref[gi] + (T)sign * (u[ii] - ref[ii]);
}

// Coarse half of a tiled prolongation: C[lz][ly][lx] = u^H - u^H_old at coarse
// cell (cx0 + lx, cy0 + ly, cz0 + lz) for lz < cz (periodic wrap; zero outside a
// Dirichlet grid).  The loop has a fixed trip count, so all its loads are
// issued before the first is needed.
template <int DIR, typename T, int CZM, int CY, int CX>
__device__ __forceinline__ void stage_coarse_diff(const Geom& gc, const T* __restrict__ uc,
                                                  const T* __restrict__ oldc, T (&C)[CZM][CY][CX], int cz,
                                                  int cx0, int cy0, int cz0) {
    constexpr int NS = (CZM * CY * CX + NT - 1) / NT;
    T v[NS];
    int li[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int e = (int)threadIdx.x + s * NT;
        const int lx = e % CX, ly = (e / CX) % CY, lz = e / (CX * CY);
        int I = cx0 + lx, J = cy0 + ly, K = cz0 + lz;
        bool ok = lz < cz;
        if (DIR) {
            ok = ok && I >= 0 && I < gc.n0 && J >= 0 && J < gc.n1 && K >= 0 && K < gc.n2;
        } else {
            I = wrapi(I, gc.n0);
            J = wrapi(J, gc.n1);
            K = wrapi(K, gc.n2);
        }
        const int64_t ci = ok ? cell_index(gc, I, J, K) : 0;
        const T a = uc[ci], b = oldc[ci];
        v[s] = ok ? a - b : T(0);
        li[s] = lz < cz ? e : -1;
    }
#pragma unroll
    for (int s = 0; s < NS; ++s)
        if (li[s] >= 0) (&C[0][0][0])[li[s]] = v[s];
}

// Fine half of a tiled prolongation u^h += P c (cell-centred trilinear, weights
// 3/4 and 1/4 per axis) once the coarse values c around the tile sit in LDS
// (C[.][.][0] is coarse cell (cx0, cy0, cz0)).  Lane = fine x within the
// 64-wide tile; wave w takes fine rows q = w, w + 4, ... of the 8 x pz rows
// (y fastest), NBAT rows per batch so that NBAT loads are in flight.
template <int NBAT, typename T, int CZM, int CY, int CX>
__device__ __forceinline__ void prolong_tile_rows(const Geom& gf, T* __restrict__ uf,
                                                  const T (&C)[CZM][CY][CX], int x0, int y0, int z0,
                                                  int cx0, int cy0, int cz0, int pz) {
    const int i = x0 + (int)(threadIdx.x & 63);
    if (i >= gf.n0) return;
    const int Ii = (i >> 1) - cx0, si = (i & 1) ? 1 : -1;
    const T a = T(0.75), b = T(0.25);
    constexpr int NW = NT / 64;
    const int nq = 8 * pz;
    for (int q0 = (int)(threadIdx.x >> 6); q0 < nq; q0 += NW * NBAT) {
        T v[NBAT];
        int64_t gi[NBAT];
        bool ok[NBAT];
#pragma unroll
        for (int u = 0; u < NBAT; ++u) {
            const int q = q0 + u * NW;
            const int j = y0 + (q & 7), k = z0 + (q >> 3);
            ok[u] = q < nq && j < gf.n1 && k < gf.n2;
            gi[u] = ok[u] ? cell_index(gf, i, j, k) : 0;
            v[u] = ok[u] ? uf[gi[u]] : T(0);
        }
#pragma unroll
        for (int u = 0; u < NBAT; ++u) {
            if (!ok[u]) continue;
            const int q = q0 + u * NW;
            const int j = y0 + (q & 7), k = z0 + (q >> 3);
            const int Jj = (j >> 1) - cy0, sj = (j & 1) ? 1 : -1;
            const int Kk = (k >> 1) - cz0, sk = (k & 1) ? 1 : -1;
            const T x00 = a * C[Kk][Jj][Ii] + b * C[Kk][Jj][Ii + si];
            const T x10 = a * C[Kk][Jj + sj][Ii] + b * C[Kk][Jj + sj][Ii + si];
            const T x01 = a * C[Kk + sk][Jj][Ii] + b * C[Kk + sk][Jj][Ii + si];
            const T x11 = a * C[Kk + sk][Jj + sj][Ii] + b * C[Kk + sk][Jj + sj][Ii + si];
            const T y0v = a * x00 + b * x10, y1v = a * x01 + b * x11;
            uf[gi[u]] = v[u] + (a * y0v + b * y1v);
        }
    }
}

static inline int grid_for(int64_t n, int cap = 65536) {
    int64_t b = (n + NT - 1) / NT;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

}  // namespace vmg
