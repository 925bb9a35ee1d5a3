// gfx950 kernels of the mixed-precision path: FP32 smoothing, restriction and
// prolongation of a correction e inside an FP64 defect-correction loop.
//
// Outer (FP64): d = L(phi) + cbar - f  (Sec. III.B/III.C operator), then phi += e.
// Inner (FP32): find e with L(phi + e) - L(phi) = -d, i.e.
//     Lap_h e - dQ(e) = r - cbar_e,     r = -d (cast to FP32),
//     dQ(e) = Q(q0 + dq) - Q(q0),       dq = alpha * Phi(2 phi~ + e, e) / h^4,
// where Phi is the symmetric bilinear form with Phi(u,u) = Sigma0(u) h^4
// (Sigma0 of the discrete Sigma_ijk at w = 1/3 without its density term), so
// Sigma0(phi+e) - Sigma0(phi) = Phi(2 phi + e, e) / h^4.  With Q(q) = 3/(4 alpha)
// (sqrt(max(D,0)) - 1), D = 1 + 8 alpha q / 3:
//     dQ = 2 dq / (s0 + s1)             if D0 >= 0 and D1 >= 0 (no cancellation)
//     dQ = 3/(4 alpha) (s1 - s0)        otherwise (the discriminant guard is active)
// with s = sqrt(max(D, 0)).  D0 comes from the FP64 state as t0 = +-sqrt(|D0|)
// (sign of D0), so the root near a vanishing discriminant is evaluated in FP64.
// dQ does not depend on e at the cell itself, so the nonlinear Gauss-Seidel
// update stays closed form: e_c <- (S_e - h^2 (dQ + r - cbar_e)) / 6.
#include <algorithm>
#include <cstring>

#include "brick.h"

namespace vmg {

// ---------------------------------------------------------------------------
// fused red-black sweep on e (same schedule and tiling as the FP64 sweep)
// ---------------------------------------------------------------------------
struct CorrArgs {
    Geom g;
    CoefF c;
    const float* ein;
    float* eout;
    const float* pt;   // phi~ (FP32 base state)
    const float* t0;
    const float* r;
    const LevelScalars* sc;   // inner cbar
    // prolongation folded into the sweep (periodic): ein += P(uc - oc) first
    Geom gc;
    const float* uc;          // null: no prolongation
    const float* oc;
    int zc, tiles_x, tiles_y;
    // Dirichlet bricks below the finest level: reference of the ghost refresh
    // (null: the ghost shell of eout is left to a separate refresh)
    const float* gref;
};

// FP32 correction policy of the fused sweep (brick.h): a cell holds (e, phi~),
// so one 8-byte LDS read gives both neighbourhoods; sources are t0 and r.
// ZERO_E: the input correction is identically zero and is not read.
template <bool ZERO_E>
struct CorrK {
    using Cell = float2;   // (e, phi~)
    using Corr = float;
    static constexpr int AHEAD = 1;   // fewer registers; measured faster than 2 here
    struct Src {
        float t0, r;
    };
    const float* __restrict__ ein;
    float* __restrict__ eout;
    const float* __restrict__ pt;
    const float* __restrict__ t0;
    const float* __restrict__ r;
    CoefF c;
    float h2_6, cb_6;   // h^2/6, h^2 cbar/6
    float kk;           // kink_k(h^2)
    Geom gc;            // folded prolongation: coarse level and its e^H, e^H_old
    const float* __restrict__ uc;
    const float* __restrict__ oc;
    const float* __restrict__ gref;

    __device__ CorrK(const CorrArgs& a, bool periodic)
        : ein(a.ein), eout(a.eout), pt(a.pt), t0(a.t0), r(a.r), c(a.c), gc(a.gc), uc(a.uc), oc(a.oc),
          gref(a.gref) {
        h2_6 = c.h2 * (1.0f / 6.0f);
        kk = kink_k(c.h2);
        cb_6 = periodic ? h2_6 * (float)a.sc->cbar : 0.0f;
    }
    static constexpr int EB = 4;
    struct InPlane {
        __amdgpu_buffer_rsrc_t e, p;
    };
    struct SrcPlane {
        __amdgpu_buffer_rsrc_t t, r;
    };
    struct OutPlane {
        __amdgpu_buffer_rsrc_t e;
    };
    __device__ InPlane in_plane(int64_t zo, bool ok) const {
        return InPlane{plane_rsrc(ZERO_E ? pt : ein, zo, EB, ok && !ZERO_E), plane_rsrc(pt, zo, EB, ok)};
    }
    __device__ SrcPlane src_plane(int64_t zo, bool ok) const {
        return SrcPlane{plane_rsrc(t0, zo, EB, ok), plane_rsrc(r, zo, EB, ok)};
    }
    __device__ OutPlane out_plane(int64_t zo, bool ok) const { return OutPlane{plane_rsrc(eout, zo, EB, ok)}; }
    __device__ float2 cell_b(const InPlane& P, int bo) const {
        return make_float2(ZERO_E ? 0.0f : buf_ld_f32(P.e, bo), buf_ld_f32(P.p, bo));
    }
    // a cell outside the grid reads t0 = 0 and r = 0; no update is formed from it
    __device__ Src src_b(const SrcPlane& S, int bo) const { return Src{buf_ld_f32(S.t, bo), buf_ld_f32(S.r, bo)}; }
    __device__ void out_b(const OutPlane& O, int bo, float2 v) const { buf_st_f32(O.e, bo, v.x); }
    struct CoarsePlane {
        __amdgpu_buffer_rsrc_t u, o;
    };
    __device__ CoarsePlane coarse_plane(int64_t zo) const {
        return CoarsePlane{plane_rsrc(uc, zo, EB, true), plane_rsrc(oc, zo, EB, true)};
    }
    __device__ float coarse_b(const CoarsePlane& C, int bo) const {
        return buf_ld_f32(C.u, bo) - buf_ld_f32(C.o, bo);
    }
    __device__ float2 add_corr(float2 u, float v) const { return make_float2(u.x + v, u.y); }
    // (the centre's phi~ travels with the red-updated cell: the black phase reads it)
    template <int W>
    __device__ float2 update(const float2* Pm, const float2* Pc, const float2* Pp, int co, int o,
                             const Src& s) const {
        NbT<float2> v;
        nb_split<W>(Pm, Pc, Pp, co, o, v);
        return update_nb(v, Pc[o], s);
    }
    // element access of the multi-sweep brick (brick_sweeps)
    __device__ float2 load_cell(int64_t i) const { return make_float2(ZERO_E ? 0.0f : ein[i], pt[i]); }
    __device__ Src load_src(int64_t i) const { return Src{t0[i], r[i]}; }
    __device__ void store_cell(int64_t i, float2 v) const { eout[i] = v.x; }
    __device__ float load_corr(int64_t i) const { return uc[i] - oc[i]; }
    // ghost gi mirrored at interior element ii (sign s) after that cell became v
    __device__ void store_ghost(int64_t gi, int64_t ii, int s, float2 v) const {
        eout[gi] = gref[gi] + (float)s * (v.x - gref[ii]);
    }
    __device__ float2 update_nb(const NbT<float2>& v, float2 centre, const Src& s) const {
        float e, D1;
        corr_new(v, s, e, D1);
        return make_float2(kink_relax(centre.x, e, D1, kk), centre.y);
    }
    // the plain update of e and the discriminant D1 of the corrected state
    __device__ void corr_new(const NbT<float2>& v, const Src& s, float& e, float& D1) const {
        NbT<float> ve, vp;
#define VMG_SPLIT(m) ve.m = v.m.x; vp.m = v.m.y;
        VMG_SPLIT(xm) VMG_SPLIT(xp) VMG_SPLIT(ym) VMG_SPLIT(yp) VMG_SPLIT(zm) VMG_SPLIT(zp)
        VMG_SPLIT(xpyp) VMG_SPLIT(xmym) VMG_SPLIT(xpym) VMG_SPLIT(xmyp)
        VMG_SPLIT(xpzp) VMG_SPLIT(xmzm) VMG_SPLIT(xpzm) VMG_SPLIT(xmzp)
        VMG_SPLIT(ypzp) VMG_SPLIT(ymzm) VMG_SPLIT(ypzm) VMG_SPLIT(ymzp)
#undef VMG_SPLIT
        float Se;
        const float dq = dq_corr(ve, vp, c.a_ih4, Se);
        const float dQ = dQ_of_d(dq, s.t0, c, D1);
        // (Se - h^2 (dQ + r - cbar)) / 6
        e = fmaf(Se, 1.0f / 6.0f, fmaf(-h2_6, dQ, fmaf(-h2_6, s.r, cb_6)));
    }
};

// PRO: the sweep starts from ein + P(uc - oc), the coarse correction prolonged
// as the planes are staged (periodic grids, even z chunks)
template <int TY, int DIR, bool ZERO_E, bool DEFER, bool PRO = false>
__global__ void __launch_bounds__(sweep_threads(TY), sweep_waves(TY, DEFER, PRO)) k_smooth_corr(CorrArgs a) {
    int b = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = b % a.tiles_x;
    b /= a.tiles_x;
    const int ty = b % a.tiles_y;
    const int ch = b / a.tiles_y;
    const int z0 = ch * a.zc;
    if (z0 >= a.g.n2) return;
    const CorrK<ZERO_E> k(a, DIR == 0);
    fused_sweep<TY, DIR, sweep_threads(TY), DEFER, PRO>(k, a.g, tx * TX, ty * TY, z0, min(z0 + a.zc, a.g.n2));
}

// S sweeps (1 or 2) of the correction on a small periodic level, one BB^3 brick
// per block (brick_sweeps); PRO adds the prolonged coarse correction first
template <int S, bool ZERO_E, bool PRO>
__global__ void __launch_bounds__(BRICK_THREADS, BRICK_WAVES) k_smooth_corr_brick(CorrArgs a) {
    const int nbx = (a.g.n0 + BB - 1) / BB, nby = (a.g.n1 + BB - 1) / BB;
    int b = xcd_remap(blockIdx.x, gridDim.x);
    const int bx = b % nbx;
    b /= nbx;
    const int by = b % nby, bz = b / nby;
    const CorrK<ZERO_E> k(a, true);
    brick_sweeps<S, PRO>(k, a.g, bx * BB, by * BB, bz * BB);
}

// persistent sweep over a (grid, tile x, tile y, z chunk) work list (Dirichlet batches)
template <int TY, bool DEFER>
__global__ void __launch_bounds__(sweep_threads(TY), sweep_waves(TY, DEFER)) k_smooth_corr_batch(CorrArgs proto, const Geom* __restrict__ geoms,
                                                          const int4* __restrict__ items, int nitems) {
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int4 w = items[it];
        CorrArgs a = proto;
        a.g = geoms[w.x];
        a.c.a_ih4 = proto.c.alpha / (float)(a.g.h * a.g.h * a.g.h * a.g.h);
        a.c.h2 = (float)(a.g.h * a.g.h);
        const int z0 = w.w * a.zc;
        const CorrK<false> k(a, false);
        fused_sweep<TY, 1, sweep_threads(TY), DEFER>(k, a.g, w.y * TX, w.z * TY, z0, min(z0 + a.zc, a.g.n2));
    }
}

// one sweep of every grid of a Dirichlet batch at one level on BB^3 bricks
// (items: grid, brick x, brick y, brick z)
template <bool GHOSTS>
__global__ void __launch_bounds__(BRICK_THREADS, BRICK_WAVES) k_smooth_corr_brick_batch(CorrArgs proto,
                                                                                        const Geom* __restrict__ geoms,
                                                                                        const int4* __restrict__ items,
                                                                                        int nitems) {
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int4 w = items[it];
        CorrArgs a = proto;
        a.g = geoms[w.x];
        a.c.a_ih4 = proto.c.alpha / (float)(a.g.h * a.g.h * a.g.h * a.g.h);
        a.c.h2 = (float)(a.g.h * a.g.h);
        const CorrK<false> k(a, false);
        brick_sweeps<1, false, 1, GHOSTS>(k, a.g, w.y * BB, w.z * BB, w.w * BB);
        __syncthreads();   // the next item's staging overwrites the LDS
    }
}

// ---------------------------------------------------------------------------
// inner residual + restriction, inner FAS rhs, prolongation (FP32 data, FP64 sums)
// ---------------------------------------------------------------------------
template <int DIR>
__device__ __forceinline__ float corr_residual(const Geom& g, const CoefF& c, const float* e,
                                               const float* pt, const float* t0, const float* r,
                                               float cb, int i, int j, int k, float inv_h2,
                                               float& dQ, float& ec, float& rv) {
    NbT<float> ve, vp;
    ec = gather_nb<DIR>(g, e, i, j, k, ve);
    gather_nb<DIR>(g, pt, i, j, k, vp);
    const int64_t gi = cell_index(g, i, j, k);
    float Se;
    const float dq = dq_corr(ve, vp, c.a_ih4, Se);
    dQ = dQ_of(dq, t0[gi], c);
    rv = r ? r[gi] : 0.0f;
    return (Se - 6.0f * ec) * inv_h2 - dQ - rv + cb;
}

template <int DIR>
__global__ void __launch_bounds__(NT) k_rr_corr(Geom gf, Geom gc, CoefF c, const float* __restrict__ e,
                                                const float* __restrict__ pt, const float* __restrict__ t0,
                                                const float* __restrict__ r, const LevelScalars* sc,
                                                float* ec, float* eold_c, float* rd_c, double* partials) {
    double acc[R_NSLOT] = {0, 0, 0, 0, 0, 0, 0};
    const float cb = DIR ? 0.0f : (float)sc->cbar;
    const float inv_h2 = 1.0f / c.h2;
    for (int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x; q < gc.ncell; q += (int64_t)gridDim.x * NT) {
        int I, J, K;
        decode(gc, q, I, J, K);
        float se = 0.0f, sd = 0.0f;
#pragma unroll
        for (int ch = 0; ch < 8; ++ch) {
            const int i = 2 * I + (ch & 1), j = 2 * J + ((ch >> 1) & 1), k = 2 * K + (ch >> 2);
            float dQ, ev, rv;
            const float d = corr_residual<DIR>(gf, c, e, pt, t0, r, cb, i, j, k, inv_h2, dQ, ev, rv);
            acc[R_D2] += (double)d * d;
            acc[R_D1] += d;
            acc[R_Q] += dQ;
            acc[R_F] += rv;
            acc[R_NONFIN] += isfinite(d) ? 0.0 : 1.0;
            se += ev;
            sd += d;
        }
        const int64_t co = cell_index(gc, I, J, K);
        ec[co] = 0.125f * se;
        eold_c[co] = 0.125f * se;
        rd_c[co] = 0.125f * sd;
    }
    block_store_partials(acc, partials);
}

template <int DIR>
__global__ void __launch_bounds__(NT) k_fas_corr(Geom g, CoefF c, const float* __restrict__ e,
                                                 const float* __restrict__ pt, const float* __restrict__ t0,
                                                 const float* __restrict__ rd, float* r, double* partials) {
    double acc[R_NSLOT] = {0, 0, 0, 0, 0, 0, 0};
    const float inv_h2 = 1.0f / c.h2;
    for (int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x; q < g.ncell; q += (int64_t)gridDim.x * NT) {
        int i, j, k;
        decode(g, q, i, j, k);
        float dQ, ev, rv;
        const float L = corr_residual<DIR>(g, c, e, pt, t0, nullptr, 0.0f, i, j, k, inv_h2, dQ, ev, rv);
        const int64_t gi = cell_index(g, i, j, k);
        const float rh = L - rd[gi];
        r[gi] = rh;
        acc[R_Q] += dQ;
        acc[R_F] += rh;
    }
    block_store_partials(acc, partials);
}

template <int DIR>
__global__ void __launch_bounds__(NT) k_prolong_corr(Geom gf, Geom gc, float* __restrict__ ef,
                                                     const float* __restrict__ ecs,
                                                     const float* __restrict__ oldc) {
    for (int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x; q < gf.ncell; q += (int64_t)gridDim.x * NT) {
        int i, j, k;
        decode(gf, q, i, j, k);
        const int I = i >> 1, J = j >> 1, K = k >> 1;
        const int si = (i & 1) ? 1 : -1, sj = (j & 1) ? 1 : -1, sk = (k & 1) ? 1 : -1;
        float acc = 0.0f;
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            int ii = I + ((m & 1) ? si : 0), jj = J + ((m & 2) ? sj : 0), kk = K + ((m & 4) ? sk : 0);
            const float w = ((m & 1) ? 0.25f : 0.75f) * ((m & 2) ? 0.25f : 0.75f) * ((m & 4) ? 0.25f : 0.75f);
            float corr;
            if (DIR) {
                if (ii < 0 || ii >= gc.n0 || jj < 0 || jj >= gc.n1 || kk < 0 || kk >= gc.n2) {
                    corr = 0.0f;
                } else {
                    const int64_t ci = cell_index(gc, ii, jj, kk);
                    corr = ecs[ci] - oldc[ci];
                }
            } else {
                ii = ii < 0 ? ii + gc.n0 : (ii >= gc.n0 ? ii - gc.n0 : ii);
                jj = jj < 0 ? jj + gc.n1 : (jj >= gc.n1 ? jj - gc.n1 : jj);
                kk = kk < 0 ? kk + gc.n2 : (kk >= gc.n2 ? kk - gc.n2 : kk);
                const int64_t ci = cell_index(gc, ii, jj, kk);
                corr = ecs[ci] - oldc[ci];
            }
            acc += w * corr;
        }
        ef[cell_index(gf, i, j, k)] += acc;
    }
}

// coarsest inner level, whole grid in LDS
template <int DIR>
__device__ __forceinline__ void coarse_corr_body(Geom g, CoefF c, float* e, float* e_also, const float* pt,
                                                 const float* t0, const float* r, int sweeps,
                                                 const float* old = nullptr) {
    constexpr int CM = 1000;
    __shared__ float se[CM], sp[CM], st[CM], sr[CM], so[CM];
    __shared__ double red[NT / 64];
    const int tid = threadIdx.x, nt = blockDim.x;
    e += g.base;
    pt += g.base;
    t0 += g.base;
    r += g.base;
    if (e_also) e_also += g.base;
    if (old) old += g.base;
    c.a_ih4 = c.alpha / (float)(g.h * g.h * g.h * g.h);
    c.h2 = (float)(g.h * g.h);
    g.off0 -= g.base;
    g.base = 0;
    for (int64_t q = tid; q < g.nstore; q += nt) {
        se[q] = e[q];
        sp[q] = pt[q];
        st[q] = t0[q];
        sr[q] = r[q];
        if (DIR && old) so[q] = old[q];
    }
    __syncthreads();
    const int64_t nghost = DIR ? ghost_count_dev(g.n0, g.n1, g.n2) : 0;
    auto refresh_ghosts = [&]() {
        if (!DIR || !old) return;
        for (int64_t q = tid; q < nghost; q += nt) {
            int i, j, k;
            ghost_coords(g.n0, g.n1, g.n2, q, i, j, k);
            int sign = 1;
            const int ir = mirror(i, g.n0, sign), jr = mirror(j, g.n1, sign), kr = mirror(k, g.n2, sign);
            const int64_t gi = cell_index(g, i, j, k), ii = cell_index(g, ir, jr, kr);
            se[gi] = so[gi] + (float)sign * (se[ii] - so[ii]);
        }
        __syncthreads();
    };
    const float h2 = c.h2;
    double sumr = 0.0;
    if (!DIR) {
        double acc = 0.0;
        for (int64_t q = tid; q < g.ncell; q += nt) {
            int i, j, k;
            decode(g, q, i, j, k);
            acc += sr[cell_index(g, i, j, k)];
        }
        acc = wave_sum(acc);
        if ((tid & 63) == 0) red[tid >> 6] = acc;
        __syncthreads();
        for (int w = 0; w < nt / 64; ++w) sumr += red[w];
        __syncthreads();
    }
    const int per = (int)((g.ncell + nt - 1) / nt);
    for (int s = 0; s < sweeps; ++s) {
        float cb = 0.0f;
        if (!DIR) {
            double acc = 0.0;
            for (int64_t q = tid; q < g.ncell; q += nt) {
                int i, j, k;
                decode(g, q, i, j, k);
                NbT<float> ve, vp;
                gather_nb<DIR>(g, se, i, j, k, ve);
                gather_nb<DIR>(g, sp, i, j, k, vp);
                float Se;
                acc += dQ_of(dq_corr(ve, vp, c.a_ih4, Se), st[cell_index(g, i, j, k)], c);
            }
            acc = wave_sum(acc);
            if ((tid & 63) == 0) red[tid >> 6] = acc;
            __syncthreads();
            double sq = 0.0;
            for (int w = 0; w < nt / 64; ++w) sq += red[w];
            cb = (float)((sumr + sq) / (double)g.ncell);
            __syncthreads();
        }
        for (int colour = 0; colour < 2; ++colour) {
            float nv[2];
            int64_t ni[2] = {-1, -1};
            for (int q = 0; q < per && q < 2; ++q) {
                const int64_t m = tid + (int64_t)q * nt;
                if (m >= g.ncell) continue;
                int i, j, k;
                decode(g, m, i, j, k);
                if (((i + j + k) & 1) != colour) continue;
                NbT<float> ve, vp;
                gather_nb<DIR>(g, se, i, j, k, ve);
                gather_nb<DIR>(g, sp, i, j, k, vp);
                const int64_t li = cell_index(g, i, j, k);
                float Se, D1;
                const float dQ = dQ_of_d(dq_corr(ve, vp, c.a_ih4, Se), st[li], c, D1);
                nv[q] = kink_relax(se[li], (Se - h2 * (dQ + sr[li] - cb)) * (1.0f / 6.0f), D1, kink_k(h2));
                ni[q] = li;
            }
            __syncthreads();
            for (int q = 0; q < 2; ++q)
                if (ni[q] >= 0) se[ni[q]] = nv[q];
            __syncthreads();
            refresh_ghosts();
        }
    }
    for (int64_t q = tid; q < g.ncell; q += nt) {
        int i, j, k;
        decode(g, q, i, j, k);
        const int64_t li = cell_index(g, i, j, k);
        e[li] = se[li];
        if (e_also) e_also[li] = se[li];
    }
    if (DIR && old)
        for (int64_t q = tid; q < nghost; q += nt) {
            int i, j, k;
            ghost_coords(g.n0, g.n1, g.n2, q, i, j, k);
            const int64_t li = cell_index(g, i, j, k);
            e[li] = se[li];
            if (e_also) e_also[li] = se[li];
        }
    __syncthreads();
}

template <int DIR>
__global__ void __launch_bounds__(NT) k_coarse_corr(Geom g, CoefF c, float* e, const float* pt,
                                                    const float* t0, const float* r, int sweeps) {
    coarse_corr_body<DIR>(g, c, e, nullptr, pt, t0, r, sweeps);
}

// coarsest inner levels of several Dirichlet grids, one block per grid; result in both e buffers
__global__ void __launch_bounds__(NT) k_coarse_corr_batch(const Geom* __restrict__ gs, CoefF c, float* e0,
                                                          float* e1, const float* pt, const float* t0,
                                                          const float* r, int sweeps, const float* old) {
    coarse_corr_body<1>(gs[blockIdx.x], c, e0, e1, pt, t0, r, sweeps, old);
}

// D0 = 1 + (8 alpha/3)(alpha Sigma0 + kappa delta) of the FP64 state (same arithmetic as nl_root)

// t0 = +-sqrt|D0| of a coarse inner level from its FP32 base state and density
template <int DIR>
__device__ __forceinline__ float base_t0_cell(const Geom& g, const Coef& c, const float* pt, const double* delta,
                                              int i, int j, int k, double inv_h4) {
    NbT<float> vf;
    gather_nb<DIR>(g, pt, i, j, k, vf);
    Nb v;
    v.xm = vf.xm; v.xp = vf.xp; v.ym = vf.ym; v.yp = vf.yp; v.zm = vf.zm; v.zp = vf.zp;
    v.xpyp = vf.xpyp; v.xmym = vf.xmym; v.xpym = vf.xpym; v.xmyp = vf.xmyp;
    v.xpzp = vf.xpzp; v.xmzm = vf.xmzm; v.xpzm = vf.xpzm; v.xmzp = vf.xmzp;
    v.ypzp = vf.ypzp; v.ymzm = vf.ymzm; v.ypzm = vf.ypzm; v.ymzp = vf.ymzp;
    const double D0 = base_discriminant(v, delta[cell_index(g, i, j, k)], c, inv_h4);
    return (float)(D0 >= 0.0 ? sqrt(D0) : -sqrt(-D0));
}

// ---------------------------------------------------------------------------
// outer FP64 pass: residual of phi, norm partials, and the FP32 inputs of the
// inner problem (phi~ = fp32(phi), t0 = +-sqrt|D0|, r = -d)
// ---------------------------------------------------------------------------
template <int DIR>
__global__ void __launch_bounds__(NT) k_cast(Geom g, Coef c, const double* __restrict__ phi,
                                             const double* __restrict__ delta, const double* __restrict__ f,
                                             const LevelScalars* sc, float* pt, float* t0, float* r,
                                             double* partials) {
    double acc[R_NSLOT] = {0, 0, 0, 0, 0, 0, 0};
    const double cb = DIR ? 0.0 : sc->cbar;
    const double inv_h2 = 1.0 / (g.h * g.h), inv_h4 = inv_h2 * inv_h2;
    for (int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x; q < g.ncell; q += (int64_t)gridDim.x * NT) {
        int i, j, k;
        decode(g, q, i, j, k);
        Nb v;
        const double pc = gather_nb<DIR>(g, phi, i, j, k, v);
        const int64_t gi = cell_index(g, i, j, k);
        double S;
        bool gd;
        const double dl = delta[gi];
        const double Q = nl_root(v, dl, c, inv_h4, S, gd);
        // D0 again for the inner problem's t0 (same arithmetic as nl_root)
        const double sx = v.xp + v.xm, sy = v.yp + v.ym, sz = v.zp + v.zm;
        const double dxy = sx - sy, dxz = sx - sz, dyz = sy - sz;
        const double bxy = (v.xpyp + v.xmym) - (v.xpym + v.xmyp);
        const double bxz = (v.xpzp + v.xmzm) - (v.xpzm + v.xmzp);
        const double byz = (v.ypzp + v.ymzm) - (v.ypzm + v.ymzp);
        const double s0 = ((dxy * dxy + dxz * dxz + dyz * dyz) * (1.0 / 3.0)
                         + (bxy * bxy + bxz * bxz + byz * byz) * 0.125) * inv_h4;
        const double D0 = 1.0 + c.c8 * (c.alpha * s0 + c.kappa * dl);
        const double fv = f ? f[gi] : 0.0;
        const double d = (S - 6.0 * pc) * inv_h2 - Q - fv + cb;
        pt[gi] = (float)pc;
        t0[gi] = (float)(D0 >= 0.0 ? sqrt(D0) : -sqrt(-D0));
        r[gi] = (float)(-d);
        acc[R_D2] += d * d;
        acc[R_D1] += d;
        acc[R_Q] += Q;
        acc[R_F] += fv;
        acc[R_PHI] += pc;
        acc[R_GUARD] += gd ? 1.0 : 0.0;
        acc[R_NONFIN] += isfinite(d) ? 0.0 : 1.0;
    }
    block_store_partials(acc, partials);
}

// base state of a coarse inner level: phi~^H = R phi~^h
__global__ void k_base_restrict(Geom gf, Geom gc, const float* pf, float* pc) {
    for (int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x; q < gc.ncell; q += (int64_t)gridDim.x * NT) {
        int I, J, K;
        decode(gc, q, I, J, K);
        float s = 0.0f;
        for (int ch = 0; ch < 8; ++ch)
            s += pf[cell_index(gf, 2 * I + (ch & 1), 2 * J + ((ch >> 1) & 1), 2 * K + (ch >> 2))];
        pc[cell_index(gc, I, J, K)] = 0.125f * s;
    }
}

// t0 of a coarse inner level from its base state and density
template <int DIR>
__global__ void k_base_t0(Geom g, Coef c, const float* pt, const double* delta, float* t0) {
    const double inv_h4 = 1.0 / (g.h * g.h * g.h * g.h);
    for (int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x; q < g.ncell; q += (int64_t)gridDim.x * NT) {
        int i, j, k;
        decode(g, q, i, j, k);
        NbT<float> vf;
        gather_nb<DIR>(g, pt, i, j, k, vf);
        const double sx = (double)vf.xp + vf.xm, sy = (double)vf.yp + vf.ym, sz = (double)vf.zp + vf.zm;
        const double dxy = sx - sy, dxz = sx - sz, dyz = sy - sz;
        const double bxy = ((double)vf.xpyp + vf.xmym) - ((double)vf.xpym + vf.xmyp);
        const double bxz = ((double)vf.xpzp + vf.xmzm) - ((double)vf.xpzm + vf.xmzp);
        const double byz = ((double)vf.ypzp + vf.ymzm) - ((double)vf.ypzm + vf.ymzp);
        const double s0 = ((dxy * dxy + dxz * dxz + dyz * dyz) * (1.0 / 3.0)
                         + (bxy * bxy + bxz * bxz + byz * byz) * 0.125) * inv_h4;
        const int64_t gi = cell_index(g, i, j, k);
        const double D0 = 1.0 + c.c8 * (c.alpha * s0 + c.kappa * delta[gi]);
        t0[gi] = (float)(D0 >= 0.0 ? sqrt(D0) : -sqrt(-D0));
    }
}

template <int DIR>
__global__ void k_update(Geom g, double* phi, const float* e) {
    for (int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x; q < g.ncell; q += (int64_t)gridDim.x * NT) {
        int i, j, k;
        decode(g, q, i, j, k);
        const int64_t gi = cell_index(g, i, j, k);
        phi[gi] += (double)e[gi];
    }
}

__global__ void k_fill_f(float* p, int64_t n, float v) {
    for (int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x; q < n; q += (int64_t)gridDim.x * NT) p[q] = v;
}

__global__ void k_cast_all(const double* src, float* dst, int64_t n) {
    for (int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x; q < n; q += (int64_t)gridDim.x * NT)
        dst[q] = (float)src[q];
}

// ---------------------------------------------------------------------------
// Tiled passes of the mixed path (same brick / z-march layout as the FP64
// residual pass: 64 x 8 x 16 bricks, one-cell LDS ring, thread = x pair of a row)
// ---------------------------------------------------------------------------
constexpr int MTY = 8, MZC = 16;

struct CastArgs {
    Geom g;
    Coef c;
    const double* phi;     // current FP64 iterate
    const float* e;        // correction to add first (UPDATE), else unused
    double* phi_out;       // phi + e (UPDATE), else unused
    const double* delta;
    const double* f;       // optional source
    const LevelScalars* sc;
    float *pt, *t0, *r;
    double* partials;
    int tiles_x, tiles_y, zc;
};

// Outer FP64 pass: phi_new = phi (+ e), d = L(phi_new) + cbar - f, norm partials,
// and the inner problem's inputs phi~ = fp32(phi_new), t0 = +-sqrt|D0|, r = -d.
template <int DIR, bool UPDATE>
__global__ void __launch_bounds__(NT) k_cast_tiled(CastArgs a) {
    constexpr int W1 = TX + 2, H1 = MTY + 2, NP1 = W1 * H1, NL1 = (NP1 + NT - 1) / NT;
    __shared__ double PH[3][H1][W1];
    const Geom& g = a.g;
    const int tid = threadIdx.x;
    int b = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = b % a.tiles_x;
    b /= a.tiles_x;
    const int ty = b % a.tiles_y;
    const int ch = b / a.tiles_y;
    const int x0 = tx * TX, y0 = ty * MTY, z0 = ch * a.zc;
    const int z1 = min(z0 + a.zc, g.n2);
    double acc[R_NSLOT] = {0, 0, 0, 0, 0, 0, 0};
    const double cb = DIR ? 0.0 : a.sc->cbar;
    const double inv_h2 = 1.0 / (g.h * g.h), inv_h4 = inv_h2 * inv_h2;
    const int m = tid & 31, r = tid >> 5;
    const int gy = y0 + r, xa = x0 + 2 * m;
    const bool row_ok = gy < g.n1;
    int off1[NL1], lds1[NL1];   // global in-plane offset, LDS word (rows split by parity)
    bool ok1[NL1];
#pragma unroll
    for (int s2 = 0; s2 < NL1; ++s2) {
        const int e = tid + s2 * NT;
        ok1[s2] = false;
        off1[s2] = 0;
        lds1[s2] = (e / W1) * W1 + split_col<W1>(e % W1);
        if (e < NP1) {
            int gx = x0 - 1 + e % W1, gyy = y0 - 1 + e / W1;
            if (DIR) {
                ok1[s2] = gx >= -1 && gx <= g.n0 && gyy >= -1 && gyy <= g.n1;
            } else {
                gx = wrapi(gx, g.n0);
                gyy = wrapi(gyy, g.n1);
                ok1[s2] = true;
            }
            off1[s2] = (int)(g.off0 + gx + (int64_t)gyy * g.sy);
        }
    }
    auto plane_off = [&](int t, bool& zok) -> int64_t {
        int gz;
        if (DIR) { gz = t; zok = t >= -1 && t <= g.n2; }
        else { gz = t < 0 ? t + g.n2 : (t >= g.n2 ? t - g.n2 : t); zok = true; }
        return (int64_t)gz * g.sz;
    };
    auto load_plane = [&](int t, double (&rr)[NL1]) {
        bool zok;
        const int64_t zo = plane_off(t, zok);
#pragma unroll
        for (int s2 = 0; s2 < NL1; ++s2) {
            const bool ok = ok1[s2] && zok && tid + s2 * NT < NP1;
            double v = ok ? a.phi[zo + off1[s2]] : 0.0;
            if (UPDATE && ok) v += (double)a.e[zo + off1[s2]];   // e is zero on ghosts
            rr[s2] = v;
        }
    };
    auto store_plane = [&](int sl, const double (&rr)[NL1]) {
        double* dst = &PH[sl][0][0];
#pragma unroll
        for (int s2 = 0; s2 < NL1; ++s2)
            if (tid + s2 * NT < NP1) dst[lds1[s2]] = rr[s2];
    };
    auto slot = [](int z) { return (z + 3) % 3; };
    auto src_fetch = [&](int t, double (&dl)[2], double (&fv)[2]) {
#pragma unroll
        for (int c2 = 0; c2 < 2; ++c2) {
            dl[c2] = 0.0;
            fv[c2] = 0.0;
            if (!row_ok || xa + c2 >= g.n0 || t >= z1) continue;
            const int64_t gi = g.off0 + xa + c2 + (int64_t)gy * g.sy + (int64_t)t * g.sz;
            dl[c2] = a.delta[gi];
            if (a.f) fv[c2] = a.f[gi];
        }
    };
    {
        double rr[NL1];
        for (int t = z0 - 1; t <= z0 + 1; ++t) {
            load_plane(t, rr);
            store_plane(slot(t), rr);
        }
    }
    double cdl[2], cfv[2];
    src_fetch(z0, cdl, cfv);
    __syncthreads();
    for (int t = z0; t < z1; ++t) {
        double nxt[NL1], ndl[2], nfv[2];
        const bool pf = t + 2 <= z1;
        if (pf) load_plane(t + 2, nxt);
        src_fetch(t + 1, ndl, nfv);
        const int sm = slot(t - 1), sc = slot(t), sp = slot(t + 1);
#pragma unroll
        for (int c2 = 0; c2 < 2; ++c2) {
            const int X = 2 * m + c2 + 1, Y = r + 1;
            if (!row_ok || xa + c2 >= g.n0) continue;
            Nb v;
            v.xm = PH[sc][Y][split_col<W1>(X - 1)]; v.xp = PH[sc][Y][split_col<W1>(X + 1)];
            v.ym = PH[sc][Y - 1][split_col<W1>(X)]; v.yp = PH[sc][Y + 1][split_col<W1>(X)];
            v.zm = PH[sm][Y][split_col<W1>(X)];     v.zp = PH[sp][Y][split_col<W1>(X)];
            v.xpyp = PH[sc][Y + 1][split_col<W1>(X + 1)]; v.xmym = PH[sc][Y - 1][split_col<W1>(X - 1)];
            v.xpym = PH[sc][Y - 1][split_col<W1>(X + 1)]; v.xmyp = PH[sc][Y + 1][split_col<W1>(X - 1)];
            v.xpzp = PH[sp][Y][split_col<W1>(X + 1)]; v.xmzm = PH[sm][Y][split_col<W1>(X - 1)];
            v.xpzm = PH[sm][Y][split_col<W1>(X + 1)]; v.xmzp = PH[sp][Y][split_col<W1>(X - 1)];
            v.ypzp = PH[sp][Y + 1][split_col<W1>(X)]; v.ymzm = PH[sm][Y - 1][split_col<W1>(X)];
            v.ypzm = PH[sm][Y + 1][split_col<W1>(X)]; v.ymzp = PH[sp][Y - 1][split_col<W1>(X)];
            const double pc = PH[sc][Y][split_col<W1>(X)];
            double S;
            bool gd;
            double t0;
            const double Q = nl_root_t0(v, cdl[c2], a.c, inv_h4, S, gd, t0);
            const double d = (S - 6.0 * pc) * inv_h2 - Q - cfv[c2] + cb;
            const int64_t gi = g.off0 + xa + c2 + (int64_t)gy * g.sy + (int64_t)t * g.sz;
            if (UPDATE) a.phi_out[gi] = pc;
            a.pt[gi] = (float)pc;
            a.t0[gi] = (float)t0;
            a.r[gi] = (float)(-d);
            acc[R_D2] += d * d;
            acc[R_D1] += d;
            acc[R_Q] += Q;
            acc[R_F] += cfv[c2];
            acc[R_PHI] += pc;
            acc[R_GUARD] += gd ? 1.0 : 0.0;
            acc[R_NONFIN] += isfinite(d) ? 0.0 : 1.0;
        }
        __syncthreads();
        if (pf) store_plane(slot(t + 2), nxt);
        cdl[0] = ndl[0]; cdl[1] = ndl[1];
        cfv[0] = nfv[0]; cfv[1] = nfv[1];
        __syncthreads();
    }
    block_store_partials(acc, a.partials);
}

struct CorrResArgs {
    Geom g, gc;
    CoefF c;
    const float* e;
    const float* pt;
    const float* t0;           // MODE 1, 3
    const float* r;            // inner rhs (MODE 1) or R d_e (MODE 2, 3)
    const LevelScalars* sc;    // inner cbar (MODE 1, periodic)
    float *ec, *eold_c, *rd_c; // MODE 1
    float* ptc;                // MODE 1: restricted base state (may be null)
    float* rout;               // MODE 2
    Coef c64;                  // MODE 2: FP64 coefficients of the base discriminant
    const double* delta;       // MODE 2: density of this level
    float* t0out;              // MODE 2: t0 of this level, computed here from phi~ and delta
    double* partials;
    int tiles_x, tiles_y, zc;
};

// MODE 1: inner residual d_e = Lap e - dQ(e) - r + cbar_e, reductions, R e -> ec, eold_c, R d_e -> rd_c
// MODE 2: coarse inner rhs rout = Lap e - dQ(e) - rd, reductions of dQ and rout; the
//         level's t0 = +-sqrt|D0| of the base state is computed here (FP64 discriminant
//         of phi~ and delta) and written for the smoother of this level
// MODE 3: as MODE 2, with the level's t0 read instead (its base state has not
//         changed since a MODE 2 pass set it)
template <int DIR, int MODE>
__global__ void __launch_bounds__(NT) k_corr_tiled(CorrResArgs a) {
    constexpr int W1 = TX + 2, H1 = MTY + 2, NP1 = W1 * H1, NL1 = (NP1 + NT - 1) / NT;
    __shared__ float2 EP[3][H1][W1];   // (e, phi~): one 8-byte read per neighbour
    const Geom& g = a.g;
    const int tid = threadIdx.x;
    int b = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = b % a.tiles_x;
    b /= a.tiles_x;
    const int ty = b % a.tiles_y;
    const int ch = b / a.tiles_y;
    const int x0 = tx * TX, y0 = ty * MTY, z0 = ch * a.zc;
    const int z1 = min(z0 + a.zc, g.n2);
    double acc[R_NSLOT] = {0, 0, 0, 0, 0, 0, 0};
    const float cb = (DIR || MODE >= 2) ? 0.0f : (float)a.sc->cbar;
    const float inv_h2 = 1.0f / a.c.h2;
    const int m = tid & 31, r = tid >> 5;
    const int gy = y0 + r, xa = x0 + 2 * m;
    const bool row_ok = gy < g.n1;
    int off1[NL1], lds1[NL1];   // global in-plane offset, LDS word (rows split by parity)
    bool ok1[NL1];
#pragma unroll
    for (int s2 = 0; s2 < NL1; ++s2) {
        const int e = tid + s2 * NT;
        ok1[s2] = false;
        off1[s2] = 0;
        lds1[s2] = (e / W1) * W1 + split_col<W1>(e % W1);
        if (e < NP1) {
            int gx = x0 - 1 + e % W1, gyy = y0 - 1 + e / W1;
            if (DIR) {
                ok1[s2] = gx >= -1 && gx <= g.n0 && gyy >= -1 && gyy <= g.n1;
            } else {
                gx = wrapi(gx, g.n0);
                gyy = wrapi(gyy, g.n1);
                ok1[s2] = true;
            }
            off1[s2] = (int)(g.off0 + gx + (int64_t)gyy * g.sy);
        }
    }
    auto plane_off = [&](int t, bool& zok) -> int64_t {
        int gz;
        if (DIR) { gz = t; zok = t >= -1 && t <= g.n2; }
        else { gz = t < 0 ? t + g.n2 : (t >= g.n2 ? t - g.n2 : t); zok = true; }
        return (int64_t)gz * g.sz;
    };
    auto load_planes = [&](int t, float (&re)[NL1], float (&rp)[NL1]) {
        bool zok;
        const int64_t zo = plane_off(t, zok);
#pragma unroll
        for (int s2 = 0; s2 < NL1; ++s2) {
            const bool ok = ok1[s2] && zok && tid + s2 * NT < NP1;
            re[s2] = ok ? a.e[zo + off1[s2]] : 0.0f;
            rp[s2] = ok ? a.pt[zo + off1[s2]] : 0.0f;
        }
    };
    auto store_planes = [&](int sl, const float (&re)[NL1], const float (&rp)[NL1]) {
        float2* d = &EP[sl][0][0];
#pragma unroll
        for (int s2 = 0; s2 < NL1; ++s2)
            if (tid + s2 * NT < NP1) d[lds1[s2]] = make_float2(re[s2], rp[s2]);
    };
    auto slot = [](int z) { return (z + 3) % 3; };
    const double inv_h4_64 = 1.0 / (g.h * g.h * g.h * g.h);
    auto src_fetch = [&](int t, float (&tt)[2], double (&dl)[2], float (&rv)[2]) {
#pragma unroll
        for (int c2 = 0; c2 < 2; ++c2) {
            tt[c2] = 1.0f;
            dl[c2] = 0.0;
            rv[c2] = 0.0f;
            if (!row_ok || xa + c2 >= g.n0 || t >= z1) continue;
            const int64_t gi = g.off0 + xa + c2 + (int64_t)gy * g.sy + (int64_t)t * g.sz;
            if (MODE == 2) dl[c2] = a.delta[gi];
            else tt[c2] = a.t0[gi];   // MODE 1, and MODE 3 (t0 of this level already set)
            rv[c2] = a.r[gi];
        }
    };
    {
        float re[NL1], rp[NL1];
        for (int t = z0 - 1; t <= z0 + 1; ++t) {
            load_planes(t, re, rp);
            store_planes(slot(t), re, rp);
        }
    }
    float ctt[2], crv[2];
    double cdl[2];
    src_fetch(z0, ctt, cdl, crv);
    __syncthreads();
    float zs_e = 0.0f, zs_d = 0.0f, zs_p = 0.0f;
    for (int t = z0; t < z1; ++t) {
        float ne[NL1], np[NL1], ntt[2], nrv[2];
        double ndl[2];
        const bool pf = t + 2 <= z1;
        if (pf) load_planes(t + 2, ne, np);
        src_fetch(t + 1, ntt, ndl, nrv);
        const int sm = slot(t - 1), sc = slot(t), sp = slot(t + 1);
        float esum = 0.0f, dsum = 0.0f, psum = 0.0f;
#pragma unroll
        for (int c2 = 0; c2 < 2; ++c2) {
            const int X = 2 * m + c2 + 1, Y = r + 1;
            if (!row_ok || xa + c2 >= g.n0) continue;
            NbT<float2> v2;
            v2.xm = EP[sc][Y][split_col<W1>(X - 1)]; v2.xp = EP[sc][Y][split_col<W1>(X + 1)]; v2.ym = EP[sc][Y - 1][split_col<W1>(X)]; v2.yp = EP[sc][Y + 1][split_col<W1>(X)];
            v2.zm = EP[sm][Y][split_col<W1>(X)]; v2.zp = EP[sp][Y][split_col<W1>(X)];
            v2.xpyp = EP[sc][Y + 1][split_col<W1>(X + 1)]; v2.xmym = EP[sc][Y - 1][split_col<W1>(X - 1)];
            v2.xpym = EP[sc][Y - 1][split_col<W1>(X + 1)]; v2.xmyp = EP[sc][Y + 1][split_col<W1>(X - 1)];
            v2.xpzp = EP[sp][Y][split_col<W1>(X + 1)]; v2.xmzm = EP[sm][Y][split_col<W1>(X - 1)]; v2.xpzm = EP[sm][Y][split_col<W1>(X + 1)]; v2.xmzp = EP[sp][Y][split_col<W1>(X - 1)];
            v2.ypzp = EP[sp][Y + 1][split_col<W1>(X)]; v2.ymzm = EP[sm][Y - 1][split_col<W1>(X)]; v2.ypzm = EP[sm][Y + 1][split_col<W1>(X)]; v2.ymzp = EP[sp][Y - 1][split_col<W1>(X)];
            NbT<float> ve, vp;
#define VMG_SPLIT(q) ve.q = v2.q.x; vp.q = v2.q.y;
            VMG_SPLIT(xm) VMG_SPLIT(xp) VMG_SPLIT(ym) VMG_SPLIT(yp) VMG_SPLIT(zm) VMG_SPLIT(zp)
            VMG_SPLIT(xpyp) VMG_SPLIT(xmym) VMG_SPLIT(xpym) VMG_SPLIT(xmyp)
            VMG_SPLIT(xpzp) VMG_SPLIT(xmzm) VMG_SPLIT(xpzm) VMG_SPLIT(xmzp)
            VMG_SPLIT(ypzp) VMG_SPLIT(ymzm) VMG_SPLIT(ypzm) VMG_SPLIT(ymzp)
#undef VMG_SPLIT
            const float2 cc = EP[sc][Y][split_col<W1>(X)];
            const float ecv = cc.x;
            float t0c = ctt[c2];
            if (MODE == 2) {
                Nb vb;
                vb.xm = vp.xm; vb.xp = vp.xp; vb.ym = vp.ym; vb.yp = vp.yp; vb.zm = vp.zm; vb.zp = vp.zp;
                vb.xpyp = vp.xpyp; vb.xmym = vp.xmym; vb.xpym = vp.xpym; vb.xmyp = vp.xmyp;
                vb.xpzp = vp.xpzp; vb.xmzm = vp.xmzm; vb.xpzm = vp.xpzm; vb.xmzp = vp.xmzp;
                vb.ypzp = vp.ypzp; vb.ymzm = vp.ymzm; vb.ypzm = vp.ypzm; vb.ymzp = vp.ymzp;
                const double D0 = base_discriminant(vb, cdl[c2], a.c64, inv_h4_64);
                t0c = (float)(D0 >= 0.0 ? sqrt(D0) : -sqrt(-D0));
                a.t0out[g.off0 + xa + c2 + (int64_t)gy * g.sy + (int64_t)t * g.sz] = t0c;
            }
            float Se;
            const float dq = dq_corr(ve, vp, a.c.a_ih4, Se);
            const float dQ = dQ_of(dq, t0c, a.c);
            const float L = (Se - 6.0f * ecv) * inv_h2 - dQ;
            if (MODE >= 2) {
                const float rh = L - crv[c2];
                a.rout[g.off0 + xa + c2 + (int64_t)gy * g.sy + (int64_t)t * g.sz] = rh;
                acc[R_Q] += dQ;
                acc[R_F] += rh;
            } else {
                const float d = L - crv[c2] + cb;
                acc[R_D2] += (double)d * d;
                acc[R_D1] += d;
                acc[R_Q] += dQ;
                acc[R_F] += crv[c2];
                acc[R_NONFIN] += isfinite(d) ? 0.0 : 1.0;
                esum += ecv;
                dsum += d;
                psum += cc.y;
            }
        }
        if (MODE == 1) {
            esum += __shfl_down(esum, 32, 64);
            dsum += __shfl_down(dsum, 32, 64);
            psum += __shfl_down(psum, 32, 64);
            if ((t & 1) == 0) {
                zs_e = esum;
                zs_d = dsum;
                zs_p = psum;
            } else if ((r & 1) == 0 && row_ok && xa < g.n0) {
                const Geom& gc = a.gc;
                const int64_t co = gc.off0 + (xa >> 1) + (int64_t)(gy >> 1) * gc.sy + (int64_t)(t >> 1) * gc.sz;
                const float re = 0.125f * (zs_e + esum);
                a.ec[co] = re;
                a.eold_c[co] = re;
                a.rd_c[co] = 0.125f * (zs_d + dsum);
                if (a.ptc) a.ptc[co] = 0.125f * (zs_p + psum);
            }
        }
        __syncthreads();
        if (pf) store_planes(slot(t + 2), ne, np);
        ctt[0] = ntt[0]; ctt[1] = ntt[1];
        cdl[0] = ndl[0]; cdl[1] = ndl[1];
        crv[0] = nrv[0]; crv[1] = nrv[1];
        __syncthreads();
    }
    block_store_partials(acc, a.partials);
}

// tiled FP32 prolongation + correction (see k_prolong_tiled)
template <int DIR>
__global__ void __launch_bounds__(NT) k_prolong_corr_tiled(Geom gf, Geom gc, float* __restrict__ ef,
                                                           const float* __restrict__ ecs,
                                                           const float* __restrict__ oldc, int tiles_x, int tiles_y,
                                                           int pzf) {
    constexpr int CX = TX / 2 + 2, CY = 8 / 2 + 2, CZM = 16 / 2 + 2;
    __shared__ float C[CZM][CY][CX];
    const int CZ = pzf / 2 + 2;
    int b = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = b % tiles_x;
    b /= tiles_x;
    const int ty = b % tiles_y;
    const int ch = b / tiles_y;
    const int x0 = tx * TX, y0 = ty * 8, z0 = ch * pzf;
    const int cx0 = x0 / 2 - 1, cy0 = y0 / 2 - 1, cz0 = z0 / 2 - 1;
    stage_coarse_diff<DIR>(gc, ecs, oldc, C, CZ, cx0, cy0, cz0);
    __syncthreads();
    prolong_tile_rows<8>(gf, ef, C, x0, y0, z0, cx0, cy0, cz0, pzf);
}

// ---------------------------------------------------------------------------
// Batched Dirichlet kernels of the mixed path (items = (grid, first cell) blocks
// of 256 cells over pooled level buffers; coefficients follow each grid's h)
// ---------------------------------------------------------------------------
__device__ __forceinline__ CoefF coef_for(CoefF c, const Geom& g) {
    c.a_ih4 = c.alpha / (float)(g.h * g.h * g.h * g.h);
    c.h2 = (float)(g.h * g.h);
    return c;
}

__global__ void __launch_bounds__(NT) k_rr_corr_batch(const Geom* __restrict__ gfs, const Geom* __restrict__ gcs,
                                                      const int2* __restrict__ items, CoefF c0,
                                                      const float* __restrict__ e, const float* __restrict__ pt,
                                                      const float* __restrict__ t0, const float* __restrict__ r,
                                                      float* ec, float* eold_c, float* rd_c) {
    // one thread per coarse cell: the children's stencils come out of two 4^3 boxes;
    // the coarse ghost shell of ec is refreshed here too
    const int2 w = items[blockIdx.x];
    const Geom gf = gfs[w.x], gc = gcs[w.x];
    const int64_t q = (int64_t)w.y + threadIdx.x;
    if (q >= gc.ncell) return;
    const CoefF c = coef_for(c0, gf);
    const float inv_h2 = 1.0f / c.h2;
    int I, J, K;
    decode(gc, q, I, J, K);
    float ub[4][4][4], pb[4][4][4];
    load_child_box(gf, e, I, J, K, ub);
    load_child_box(gf, pt, I, J, K, pb);
    float se = 0.0f, sd = 0.0f;
#pragma unroll
    for (int ch = 0; ch < 8; ++ch) {
        const int a = ch & 1, b = (ch >> 1) & 1, z = ch >> 2;
        NbT<float> ve, vp;
        const float ev = box_nb(ub, a, b, z, ve);
        box_nb(pb, a, b, z, vp);
        const int64_t gi = cell_index(gf, 2 * I + a, 2 * J + b, 2 * K + z);
        float Se;
        const float dq = dq_corr(ve, vp, c.a_ih4, Se);
        const float dQ = dQ_of(dq, t0[gi], c);
        sd += (Se - 6.0f * ev) * inv_h2 - dQ - (r ? r[gi] : 0.0f);
        se += ev;
    }
    const int64_t co = cell_index(gc, I, J, K);
    ec[co] = 0.125f * se;
    eold_c[co] = 0.125f * se;
    rd_c[co] = 0.125f * sd;
    copy_ghosts_near(gc, ec, eold_c, I, J, K);
}

__global__ void __launch_bounds__(NT) k_fas_corr_batch(const Geom* __restrict__ gs, const int2* __restrict__ items,
                                                       CoefF c0, const float* __restrict__ e,
                                                       const float* __restrict__ pt, const float* __restrict__ t0,
                                                       const float* __restrict__ rd, float* r) {
    const int2 w = items[blockIdx.x];
    const Geom g = gs[w.x];
    const int64_t q = (int64_t)w.y + threadIdx.x;
    if (q >= g.ncell) return;
    const CoefF c = coef_for(c0, g);
    int i, j, k;
    decode(g, q, i, j, k);
    float dQ, ev, rv;
    const float L = corr_residual<1>(g, c, e, pt, t0, nullptr, 0.0f, i, j, k, 1.0f / c.h2, dQ, ev, rv);
    const int64_t gi = cell_index(g, i, j, k);
    r[gi] = L - rd[gi];
}

// items: 256-cell blocks of the coarse level; each thread adds the prolonged
// correction to the 8 children of its coarse cell
__global__ void __launch_bounds__(NT) k_prolong_corr_batch(const Geom* __restrict__ gfs, const Geom* __restrict__ gcs,
                                                           const int2* __restrict__ items, float* __restrict__ ef,
                                                           const float* __restrict__ ecs,
                                                           const float* __restrict__ oldc) {
    const int2 w = items[blockIdx.x];
    const Geom gf = gfs[w.x], gc = gcs[w.x];
    const int64_t q = (int64_t)w.y + threadIdx.x;
    if (q >= gc.ncell) return;
    int I, J, K;
    decode(gc, q, I, J, K);
    prolong_children(gf, gc, ef, ecs, oldc, I, J, K);
}

__global__ void __launch_bounds__(ITEM_LANES) k_cast_batch(const Geom* __restrict__ gs,
                                                           const int2* __restrict__ items, Coef c,
                                                           const double* __restrict__ phi,
                                                           const double* __restrict__ delta,
                                                           const double* __restrict__ f, float* pt, float* t0,
                                                           float* r, double* partials) {
    double acc[R_NSLOT] = {0, 0, 0, 0, 0, 0, 0};
    const int2 w = items[blockIdx.x];
    const Geom g = gs[w.x];
    const double inv_h2 = 1.0 / (g.h * g.h), inv_h4 = inv_h2 * inv_h2;
#pragma unroll
    for (int m = 0; m < ITEM_CELLS / ITEM_LANES; ++m) {
        const int64_t q = (int64_t)w.y + threadIdx.x + m * ITEM_LANES;
        if (q >= g.ncell) break;
        int i, j, k;
        decode(g, q, i, j, k);
        Nb v;
        const double pc = gather_nb<1>(g, phi, i, j, k, v);
        const int64_t gi = cell_index(g, i, j, k);
        double S;
        bool gd;
        const double dl = delta[gi];
        const double Q = nl_root(v, dl, c, inv_h4, S, gd);
        const double D0 = base_discriminant(v, dl, c, inv_h4);
        const double fv = f ? f[gi] : 0.0;
        const double d = (S - 6.0 * pc) * inv_h2 - Q - fv;
        pt[gi] = (float)pc;
        t0[gi] = (float)(D0 >= 0.0 ? sqrt(D0) : -sqrt(-D0));
        r[gi] = (float)(-d);
        acc[R_D2] += d * d;
        acc[R_D1] += d;
        acc[R_Q] += Q;
        acc[R_F] += fv;
        acc[R_PHI] += pc;
        acc[R_GUARD] += gd ? 1.0 : 0.0;
        acc[R_NONFIN] += isfinite(d) ? 0.0 : 1.0;
    }
    wave_store_partials(acc, partials);
}

__global__ void k_base_restrict_batch(const Geom* __restrict__ gfs, const Geom* __restrict__ gcs,
                                      const int2* __restrict__ items, const float* pf, float* pc) {
    const int2 w = items[blockIdx.x];
    const Geom gf = gfs[w.x], gc = gcs[w.x];
    const int64_t q = (int64_t)w.y + threadIdx.x;
    if (q >= gc.ncell) return;
    int I, J, K;
    decode(gc, q, I, J, K);
    float s = 0.0f;
    for (int ch = 0; ch < 8; ++ch)
        s += pf[cell_index(gf, 2 * I + (ch & 1), 2 * J + ((ch >> 1) & 1), 2 * K + (ch >> 2))];
    pc[cell_index(gc, I, J, K)] = 0.125f * s;
}

__global__ void k_base_t0_batch(const Geom* __restrict__ gs, const int2* __restrict__ items, Coef c,
                                const float* pt, const double* delta, float* t0) {
    const int2 w = items[blockIdx.x];
    const Geom g = gs[w.x];
    const int64_t q = (int64_t)w.y + threadIdx.x;
    if (q >= g.ncell) return;
    const double inv_h4 = 1.0 / (g.h * g.h * g.h * g.h);
    int i, j, k;
    decode(g, q, i, j, k);
    t0[cell_index(g, i, j, k)] = base_t0_cell<1>(g, c, pt, delta, i, j, k, inv_h4);
}

__global__ void k_update_batch(const Geom* __restrict__ gs, const int2* __restrict__ items, double* phi,
                               const float* e) {
    const int2 w = items[blockIdx.x];
    const Geom g = gs[w.x];
    const int64_t q = (int64_t)w.y + threadIdx.x;
    if (q >= g.ncell) return;
    int i, j, k;
    decode(g, q, i, j, k);
    const int64_t gi = cell_index(g, i, j, k);
    phi[gi] += (double)e[gi];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int TY, int DIR>
static hipError_t corr_launch(const CorrArgs& a, bool zero_in, bool defer, hipStream_t s) {
    const dim3 nb(a.tiles_x * a.tiles_y * ((a.g.n2 + a.zc - 1) / a.zc));
    if (!DIR && a.uc && !zero_in) {
        if (defer) hipLaunchKernelGGL((k_smooth_corr<TY, 0, false, true, true>), nb, dim3(sweep_threads(TY)), 0, s, a);
        else hipLaunchKernelGGL((k_smooth_corr<TY, 0, false, false, true>), nb, dim3(sweep_threads(TY)), 0, s, a);
        return hipGetLastError();
    }
    if (zero_in && defer) hipLaunchKernelGGL((k_smooth_corr<TY, DIR, true, true>), nb, dim3(sweep_threads(TY)), 0, s, a);
    else if (zero_in) hipLaunchKernelGGL((k_smooth_corr<TY, DIR, true, false>), nb, dim3(sweep_threads(TY)), 0, s, a);
    else if (defer) hipLaunchKernelGGL((k_smooth_corr<TY, DIR, false, true>), nb, dim3(sweep_threads(TY)), 0, s, a);
    else hipLaunchKernelGGL((k_smooth_corr<TY, DIR, false, false>), nb, dim3(sweep_threads(TY)), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_smooth_corr(const Geom& g, const CoefF& c, const float* ein, float* eout,
                              const float* pt, const float* t0, const float* r, const LevelScalars* sc,
                              SmoothCfg cfg, hipStream_t s, bool zero_in, const ProlongInF* pro, int nsweeps) {
    CorrArgs a;
    std::memset(&a, 0, sizeof(a));
    a.g = g; a.c = c; a.ein = ein; a.eout = eout; a.pt = pt; a.t0 = t0; a.r = r; a.sc = sc;
    if (cfg.pipe == PIPE_BRICK) {
        // periodic levels, one or two sweeps
        if (g.dir || nsweeps < 1 || nsweeps > 2) return hipErrorInvalidValue;
        if (pro) {
            if (zero_in || !can_fold_prolong(g, pro->gc, 2)) return hipErrorInvalidValue;
            a.gc = pro->gc;
            a.uc = pro->uc;
            a.oc = pro->oc;
        }
        const dim3 nb(((g.n0 + BB - 1) / BB) * ((g.n1 + BB - 1) / BB) * ((g.n2 + BB - 1) / BB));
        const dim3 nt(BRICK_THREADS);
#define VMG_CORR_BRICK(S)                                                                                  \
    do {                                                                                                   \
        if (pro) hipLaunchKernelGGL((k_smooth_corr_brick<S, false, true>), nb, nt, 0, s, a);               \
        else if (zero_in) hipLaunchKernelGGL((k_smooth_corr_brick<S, true, false>), nb, nt, 0, s, a);      \
        else hipLaunchKernelGGL((k_smooth_corr_brick<S, false, false>), nb, nt, 0, s, a);                  \
    } while (0)
        if (nsweeps == 2) VMG_CORR_BRICK(2);
        else VMG_CORR_BRICK(1);
#undef VMG_CORR_BRICK
        return hipGetLastError();
    }
    if (nsweeps != 1) return hipErrorInvalidValue;
    a.zc = cfg.zc > 0 ? cfg.zc : 16;
    if (pro) {
        if (zero_in || !can_fold_prolong(g, pro->gc, a.zc)) return hipErrorInvalidValue;
        a.gc = pro->gc;
        a.uc = pro->uc;
        a.oc = pro->oc;
    }
    a.tiles_x = (g.n0 + TX - 1) / TX;
    a.tiles_y = (g.n1 + cfg.ty - 1) / cfg.ty;
    const bool d = cfg.pipe != 0;
    if (g.dir) {
        if (cfg.ty == 4) return corr_launch<4, 1>(a, zero_in, d, s);
        if (cfg.ty == 16) return corr_launch<16, 1>(a, zero_in, d, s);
        if (cfg.ty == 12) return corr_launch<12, 1>(a, zero_in, d, s);
        return corr_launch<8, 1>(a, zero_in, d, s);
    }
    if (cfg.ty == 4) return corr_launch<4, 0>(a, zero_in, d, s);
    if (cfg.ty == 16) return corr_launch<16, 0>(a, zero_in, d, s);
    if (cfg.ty == 12) return corr_launch<12, 0>(a, zero_in, d, s);
    return corr_launch<8, 0>(a, zero_in, d, s);
}

static void corr_tiles(const Geom& g, int& tx, int& ty, int& zc, int& nb) {
    tx = (g.n0 + TX - 1) / TX;
    ty = (g.n1 + MTY - 1) / MTY;
    zc = level_zc((int64_t)tx * ty, g.n2, 32);
    nb = tx * ty * ((g.n2 + zc - 1) / zc);
}

hipError_t launch_rr_corr(const Geom& gf, const Geom& gc, const CoefF& c, const float* e, const float* pt,
                          const float* t0, const float* r, const LevelScalars* sc, float* ec, float* eold_c,
                          float* rd_c, float* ptc, double* partials, int* nblocks_out, hipStream_t s) {
    CorrResArgs a;
    std::memset(&a, 0, sizeof(a));
    a.g = gf; a.gc = gc; a.c = c; a.e = e; a.pt = pt; a.t0 = t0; a.r = r; a.sc = sc;
    a.ec = ec; a.eold_c = eold_c; a.rd_c = rd_c; a.ptc = ptc; a.partials = partials;
    int nb;
    corr_tiles(gf, a.tiles_x, a.tiles_y, a.zc, nb);
    *nblocks_out = nb;
    if (gf.dir)
        hipLaunchKernelGGL((k_corr_tiled<1, 1>), dim3(nb), dim3(NT), 0, s, a);
    else
        hipLaunchKernelGGL((k_corr_tiled<0, 1>), dim3(nb), dim3(NT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fas_corr(const Geom& g, const CoefF& c, const Coef& c64, const double* delta, const float* e,
                           const float* pt, float* t0, const float* rd, float* r, double* partials,
                           int* nblocks_out, hipStream_t s, bool fresh_base) {
    CorrResArgs a;
    std::memset(&a, 0, sizeof(a));
    a.g = g; a.c = c; a.c64 = c64; a.delta = delta; a.e = e; a.pt = pt; a.t0out = t0; a.r = rd; a.rout = r;
    a.t0 = t0;
    a.partials = partials;
    int nb;
    corr_tiles(g, a.tiles_x, a.tiles_y, a.zc, nb);
    *nblocks_out = nb;
    if (g.dir) {
        if (fresh_base) hipLaunchKernelGGL((k_corr_tiled<1, 2>), dim3(nb), dim3(NT), 0, s, a);
        else hipLaunchKernelGGL((k_corr_tiled<1, 3>), dim3(nb), dim3(NT), 0, s, a);
    } else {
        if (fresh_base) hipLaunchKernelGGL((k_corr_tiled<0, 2>), dim3(nb), dim3(NT), 0, s, a);
        else hipLaunchKernelGGL((k_corr_tiled<0, 3>), dim3(nb), dim3(NT), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_prolong_corr(const Geom& gf, const Geom& gc, float* ef, const float* ec, const float* eold_c,
                               hipStream_t s) {
    const int tx = (gf.n0 + TX - 1) / TX, ty = (gf.n1 + 7) / 8;
    const int pz = level_zc((int64_t)tx * ty, gf.n2, 16);
    const int nb = tx * ty * ((gf.n2 + pz - 1) / pz);
    if (gf.dir)
        hipLaunchKernelGGL(k_prolong_corr_tiled<1>, dim3(nb), dim3(NT), 0, s, gf, gc, ef, ec, eold_c, tx, ty, pz);
    else
        hipLaunchKernelGGL(k_prolong_corr_tiled<0>, dim3(nb), dim3(NT), 0, s, gf, gc, ef, ec, eold_c, tx, ty, pz);
    return hipGetLastError();
}

hipError_t launch_cast_update(const Geom& g, const Coef& c, const double* phi, const float* e, double* phi_out,
                              const double* delta, const double* f, const LevelScalars* sc, float* pt, float* t0,
                              float* r, double* partials, int* nblocks_out, hipStream_t s) {
    CastArgs a;
    std::memset(&a, 0, sizeof(a));
    a.g = g; a.c = c; a.phi = phi; a.e = e; a.phi_out = phi_out; a.delta = delta; a.f = f; a.sc = sc;
    a.pt = pt; a.t0 = t0; a.r = r; a.partials = partials;
    int nb;
    corr_tiles(g, a.tiles_x, a.tiles_y, a.zc, nb);
    *nblocks_out = nb;
    const bool up = e != nullptr;
    if (g.dir) {
        if (up) hipLaunchKernelGGL((k_cast_tiled<1, true>), dim3(nb), dim3(NT), 0, s, a);
        else hipLaunchKernelGGL((k_cast_tiled<1, false>), dim3(nb), dim3(NT), 0, s, a);
    } else {
        if (up) hipLaunchKernelGGL((k_cast_tiled<0, true>), dim3(nb), dim3(NT), 0, s, a);
        else hipLaunchKernelGGL((k_cast_tiled<0, false>), dim3(nb), dim3(NT), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_coarse_corr(const Geom& g, const CoefF& c, float* e, const float* pt, const float* t0,
                              const float* r, int sweeps, hipStream_t s) {
    if (g.nstore > 1000 || g.ncell > 2 * NT) return hipErrorInvalidValue;
    const int nt = g.ncell <= 128 ? 64 : NT;
    if (g.dir)
        hipLaunchKernelGGL(k_coarse_corr<1>, dim3(1), dim3(nt), 0, s, g, c, e, pt, t0, r, sweeps);
    else
        hipLaunchKernelGGL(k_coarse_corr<0>, dim3(1), dim3(nt), 0, s, g, c, e, pt, t0, r, sweeps);
    return hipGetLastError();
}

hipError_t launch_cast(const Geom& g, const Coef& c, const double* phi, const double* delta, const double* f,
                       const LevelScalars* sc, float* pt, float* t0, float* r, double* partials,
                       int* nblocks_out, hipStream_t s) {
    const int nb = grid_for(g.ncell, 2048);
    if (g.dir)
        hipLaunchKernelGGL(k_cast<1>, dim3(nb), dim3(NT), 0, s, g, c, phi, delta, f, sc, pt, t0, r, partials);
    else
        hipLaunchKernelGGL(k_cast<0>, dim3(nb), dim3(NT), 0, s, g, c, phi, delta, f, sc, pt, t0, r, partials);
    *nblocks_out = nb;
    return hipGetLastError();
}

hipError_t launch_base_restrict(const Geom& gf, const Geom& gc, const float* pf, float* pc, hipStream_t s) {
    hipLaunchKernelGGL(k_base_restrict, dim3(grid_for(gc.ncell)), dim3(NT), 0, s, gf, gc, pf, pc);
    return hipGetLastError();
}

hipError_t launch_base_t0(const Geom& g, const Coef& c, const float* pt, const double* delta, float* t0,
                          hipStream_t s) {
    if (g.dir)
        hipLaunchKernelGGL(k_base_t0<1>, dim3(grid_for(g.ncell)), dim3(NT), 0, s, g, c, pt, delta, t0);
    else
        hipLaunchKernelGGL(k_base_t0<0>, dim3(grid_for(g.ncell)), dim3(NT), 0, s, g, c, pt, delta, t0);
    return hipGetLastError();
}

hipError_t launch_update(const Geom& g, double* phi, const float* e, hipStream_t s) {
    if (g.dir)
        hipLaunchKernelGGL(k_update<1>, dim3(grid_for(g.ncell)), dim3(NT), 0, s, g, phi, e);
    else
        hipLaunchKernelGGL(k_update<0>, dim3(grid_for(g.ncell)), dim3(NT), 0, s, g, phi, e);
    return hipGetLastError();
}

hipError_t launch_fill_f(float* p, int64_t n, float v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_f, dim3(grid_for(n)), dim3(NT), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_cast_all(const double* src, float* dst, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_cast_all, dim3(grid_for(n)), dim3(NT), 0, s, src, dst, n);
    return hipGetLastError();
}

// ---- batched launchers (Dirichlet batches) -------------------------------------
hipError_t launch_smooth_corr_batch(const CoefF& c, const float* ein, float* eout, const float* pt, const float* t0,
                                    const float* r, SmoothCfg cfg, const Geom* geoms, const int4* items, int nitems,
                                    int max_blocks, hipStream_t s, const float* gref) {
    if (nitems <= 0) return hipSuccess;
    CorrArgs a;
    std::memset(&a, 0, sizeof(a));
    a.c = c; a.ein = ein; a.eout = eout; a.pt = pt; a.t0 = t0; a.r = r; a.sc = nullptr;
    a.zc = cfg.zc > 0 ? cfg.zc : 16;
    const dim3 nb(std::min(nitems, max_blocks));
    if (cfg.pipe == PIPE_BRICK) {
        a.gref = gref;
        if (gref) hipLaunchKernelGGL((k_smooth_corr_brick_batch<true>), nb, dim3(BRICK_THREADS), 0, s, a, geoms, items, nitems);
        else hipLaunchKernelGGL((k_smooth_corr_brick_batch<false>), nb, dim3(BRICK_THREADS), 0, s, a, geoms, items, nitems);
        return hipGetLastError();
    }
    if (gref) return hipErrorInvalidValue;   // the march leaves the ghosts to a separate refresh
    const bool d = cfg.pipe != 0;
#define VMG_CORR_BATCH(T)                                                                                   \
    do {                                                                                                   \
        if (d) hipLaunchKernelGGL((k_smooth_corr_batch<T, true>), nb, dim3(sweep_threads(T)), 0, s, a, geoms, items, nitems); \
        else hipLaunchKernelGGL((k_smooth_corr_batch<T, false>), nb, dim3(sweep_threads(T)), 0, s, a, geoms, items, nitems);  \
    } while (0)
    if (cfg.ty == 4) VMG_CORR_BATCH(4);
    else if (cfg.ty == 16) VMG_CORR_BATCH(16);
    else if (cfg.ty == 12) VMG_CORR_BATCH(12);
    else VMG_CORR_BATCH(8);
#undef VMG_CORR_BATCH
    return hipGetLastError();
}

hipError_t launch_rr_corr_batch(const Geom* gfs, const Geom* gcs, const int2* items, int nitems, const CoefF& c,
                                const float* e, const float* pt, const float* t0, const float* r, float* ec,
                                float* eold_c, float* rd_c, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rr_corr_batch, dim3(nitems), dim3(NT), 0, s, gfs, gcs, items, c, e, pt, t0, r, ec, eold_c,
                       rd_c);
    return hipGetLastError();
}

hipError_t launch_fas_corr_batch(const Geom* gs, const int2* items, int nitems, const CoefF& c, const float* e,
                                 const float* pt, const float* t0, const float* rd, float* r, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fas_corr_batch, dim3(nitems), dim3(NT), 0, s, gs, items, c, e, pt, t0, rd, r);
    return hipGetLastError();
}

hipError_t launch_prolong_corr_batch(const Geom* gfs, const Geom* gcs, const int2* items, int nitems, float* ef,
                                     const float* ec, const float* eold_c, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_prolong_corr_batch, dim3(nitems), dim3(NT), 0, s, gfs, gcs, items, ef, ec, eold_c);
    return hipGetLastError();
}

hipError_t launch_coarse_corr_batch(const Geom* gs, int ngrids, const CoefF& c, float* e0, float* e1,
                                    const float* pt, const float* t0, const float* r, int sweeps, const float* old,
                                    hipStream_t s) {
    if (ngrids <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_coarse_corr_batch, dim3(ngrids), dim3(NT), 0, s, gs, c, e0, e1, pt, t0, r, sweeps, old);
    return hipGetLastError();
}

hipError_t launch_cast_batch(const Geom* gs, const int2* items, int nitems, const Coef& c, const double* phi,
                             const double* delta, const double* f, float* pt, float* t0, float* r,
                             double* partials, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cast_batch, dim3(nitems), dim3(ITEM_LANES), 0, s, gs, items, c, phi, delta, f, pt, t0, r, partials);
    return hipGetLastError();
}

hipError_t launch_base_restrict_batch(const Geom* gfs, const Geom* gcs, const int2* items, int nitems,
                                      const float* pf, float* pc, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_base_restrict_batch, dim3(nitems), dim3(NT), 0, s, gfs, gcs, items, pf, pc);
    return hipGetLastError();
}

hipError_t launch_base_t0_batch(const Geom* gs, const int2* items, int nitems, const Coef& c, const float* pt,
                                const double* delta, float* t0, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_base_t0_batch, dim3(nitems), dim3(NT), 0, s, gs, items, c, pt, delta, t0);
    return hipGetLastError();
}

hipError_t launch_update_batch(const Geom* gs, const int2* items, int nitems, double* phi, const float* e,
                               hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_update_batch, dim3(nitems), dim3(NT), 0, s, gs, items, phi, e);
    return hipGetLastError();
}

}  // namespace vmg
