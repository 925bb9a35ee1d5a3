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
#include "device_common.h"

namespace vmg {

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
    const float ph = (dxy_w * dxy_e + dxz_w * dxz_e + dyz_w * dyz_e) * (1.0f / 3.0f)
                   + (bxy_w * bxy_e + bxz_w * bxz_e + byz_w * byz_e) * 0.125f;
    return a_ih4 * ph;
}

__device__ __forceinline__ float dQ_of(float dq, float t0, const CoefF& c) {
    const float D0 = t0 >= 0.0f ? t0 * t0 : -t0 * t0;
    const float s0 = fmaxf(t0, 0.0f);
    const float D1 = D0 + c.c8 * dq;
    const float s1 = __builtin_amdgcn_sqrtf(fmaxf(D1, 0.0f));
    if (D0 >= 0.0f && D1 >= 0.0f) {
        const float den = s0 + s1;
        return den > 0.0f ? 2.0f * dq * __builtin_amdgcn_rcpf(den) : 0.0f;
    }
    return c.a34 * (s1 - s0);
}

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
    int zc, tiles_x, tiles_y;
};

template <int TY, int DIR>
__global__ void __launch_bounds__(NT) k_smooth_corr(CorrArgs a) {
    constexpr int W2 = TX + 4, H2 = TY + 4, W1 = TX + 2, H1 = TY + 2;
    constexpr int NP2 = W2 * H2, NP1 = W1 * H1;
    constexpr int NL2 = (NP2 + NT - 1) / NT, NL1 = (NP1 + NT - 1) / NT;
    constexpr int RH = W1 / 2;
    constexpr int BH = TX / 2;
    __shared__ float E0[3][H2][W2];    // e^0, ring 2
    __shared__ float PT2[3][H2][W2];   // phi~, ring 2
    __shared__ float E1[3][H1][W1];    // e^1 (red computed, black copied), ring 1
    __shared__ float PT1[3][H1][W1];   // phi~ copy, ring 1
    __shared__ float TT[3][H1][W1];    // t0, ring 1
    __shared__ float RR[3][H1][W1];    // r, ring 1

    const Geom& g = a.g;
    const int tid = threadIdx.x;
    int b = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = b % a.tiles_x;
    b /= a.tiles_x;
    const int ty = b % a.tiles_y;
    const int ch = b / a.tiles_y;
    const int x0 = tx * TX, y0 = ty * TY, z0 = ch * a.zc;
    const int z1 = min(z0 + a.zc, g.n2);
    if (z0 >= g.n2) return;
    const float h2 = a.c.h2;
    const float cb = DIR ? 0.0f : (float)a.sc->cbar;

    int off2[NL2], off1[NL1];
    bool ok2[NL2], ok1[NL1];
#pragma unroll
    for (int s = 0; s < NL2; ++s) {
        const int e = tid + s * NT;
        ok2[s] = false;
        off2[s] = 0;
        if (e < NP2) {
            int gx = x0 - 2 + e % W2, gy = y0 - 2 + e / W2;
            if (DIR) {
                ok2[s] = gx >= -1 && gx <= g.n0 && gy >= -1 && gy <= g.n1;
            } else {
                gx = wrapi(gx, g.n0);
                gy = wrapi(gy, g.n1);
                ok2[s] = true;
            }
            off2[s] = (int)(g.off0 + gx + (int64_t)gy * g.sy);
        }
    }
#pragma unroll
    for (int s = 0; s < NL1; ++s) {
        const int e = tid + s * NT;
        ok1[s] = false;
        off1[s] = 0;
        if (e < NP1) {
            int gx = x0 - 1 + e % W1, gy = y0 - 1 + e / W1;
            if (DIR) {
                ok1[s] = gx >= 0 && gx < g.n0 && gy >= 0 && gy < g.n1;
            } else {
                gx = wrapi(gx, g.n0);
                gy = wrapi(gy, g.n1);
                ok1[s] = true;
            }
            off1[s] = (int)(g.off0 + gx + (int64_t)gy * g.sy);
        }
    }
    auto zoff = [&](int t, bool& zok, bool interior_only) -> int64_t {
        int gz;
        if (DIR) { gz = t; zok = interior_only ? (t >= 0 && t < g.n2) : (t >= -1 && t <= g.n2); }
        else { gz = wrapi(t, g.n2); zok = true; }
        return (int64_t)gz * g.sz;
    };
    auto load2 = [&](const float* src, int t, float (&r)[NL2]) {
        bool zok;
        const int64_t zo = zoff(t, zok, false);
#pragma unroll
        for (int s = 0; s < NL2; ++s) r[s] = (ok2[s] && zok && tid + s * NT < NP2) ? src[zo + off2[s]] : 0.0f;
    };
    auto load1 = [&](const float* src, int t, float (&r)[NL1]) {
        bool zok;
        const int64_t zo = zoff(t, zok, true);
#pragma unroll
        for (int s = 0; s < NL1; ++s) r[s] = (ok1[s] && zok && tid + s * NT < NP1) ? src[zo + off1[s]] : 0.0f;
    };
    auto store2 = [&](float* dst, const float (&r)[NL2]) {
#pragma unroll
        for (int s = 0; s < NL2; ++s)
            if (tid + s * NT < NP2) dst[tid + s * NT] = r[s];
    };
    auto store1 = [&](float* dst, const float (&r)[NL1]) {
#pragma unroll
        for (int s = 0; s < NL1; ++s)
            if (tid + s * NT < NP1) dst[tid + s * NT] = r[s];
    };
    auto slot = [](int z) { return (z + 3) % 3; };

    {
        float r2[NL2], r1[NL1];
        for (int t = z0 - 2; t <= z0; ++t) {
            load2(a.ein, t, r2);
            store2(&E0[slot(t)][0][0], r2);
            load2(a.pt, t, r2);
            store2(&PT2[slot(t)][0][0], r2);
        }
        load1(a.t0, z0 - 1, r1);
        store1(&TT[slot(z0 - 1)][0][0], r1);
        load1(a.r, z0 - 1, r1);
        store1(&RR[slot(z0 - 1)][0][0], r1);
    }
    __syncthreads();

    for (int t = z0; t <= z1 + 1; ++t) {
        float ne[NL2], np[NL2], nt[NL1], nr[NL1];
        const bool pf2 = t + 1 <= z1 + 1, pf1 = t <= z1;
        if (pf2) {
            load2(a.ein, t + 1, ne);
            load2(a.pt, t + 1, np);
        }
        if (pf1) {
            load1(a.t0, t, nt);
            load1(a.r, t, nr);
        }
        {
            const int p = t - 1;
            const float(*Em)[W2] = E0[slot(p - 1)];
            const float(*Ec)[W2] = E0[slot(p)];
            const float(*Ep)[W2] = E0[slot(p + 1)];
            const float(*Pm)[W2] = PT2[slot(p - 1)];
            const float(*Pc)[W2] = PT2[slot(p)];
            const float(*Pp)[W2] = PT2[slot(p + 1)];
            const float(*Tc)[W1] = TT[slot(p)];
            const float(*Rc)[W1] = RR[slot(p)];
            float(*Q1)[W1] = E1[slot(p)];
            float(*C1)[W1] = PT1[slot(p)];
            const bool pzok = DIR ? (p >= 0 && p < g.n2) : true;
            for (int e = tid; e < RH * H1; e += NT) {
                const int r = e / RH, m = e - r * RH;
                const int gy = y0 - 1 + r;
                const int odd = (gy + p + 1) & 1;
                const int lx = 2 * m + odd, lb = 2 * m + 1 - odd;
                const int gx = x0 - 1 + lx;
                const int X = lx + 1, Y = r + 1;
                bool interior = true;
                if (DIR) interior = pzok && gx >= 0 && gx < g.n0 && gy >= 0 && gy < g.n1;
                float val = Ec[Y][X];
                if (interior) {
                    NbT<float> ve, vp;
#define LOADNB(v, Pm_, Pc_, Pp_)                                                        \
    v.xm = Pc_[Y][X - 1]; v.xp = Pc_[Y][X + 1]; v.ym = Pc_[Y - 1][X]; v.yp = Pc_[Y + 1][X]; \
    v.zm = Pm_[Y][X]; v.zp = Pp_[Y][X];                                                 \
    v.xpyp = Pc_[Y + 1][X + 1]; v.xmym = Pc_[Y - 1][X - 1];                             \
    v.xpym = Pc_[Y - 1][X + 1]; v.xmyp = Pc_[Y + 1][X - 1];                             \
    v.xpzp = Pp_[Y][X + 1]; v.xmzm = Pm_[Y][X - 1]; v.xpzm = Pm_[Y][X + 1]; v.xmzp = Pp_[Y][X - 1]; \
    v.ypzp = Pp_[Y + 1][X]; v.ymzm = Pm_[Y - 1][X]; v.ypzm = Pm_[Y + 1][X]; v.ymzp = Pp_[Y - 1][X];
                    LOADNB(ve, Em, Ec, Ep)
                    LOADNB(vp, Pm, Pc, Pp)
                    float Se;
                    const float dq = dq_corr(ve, vp, a.c.a_ih4, Se);
                    const float dQ = dQ_of(dq, Tc[r][lx], a.c);
                    val = (Se - h2 * (dQ + Rc[r][lx] - cb)) * (1.0f / 6.0f);
                }
                Q1[r][lx] = val;
                Q1[r][lb] = Ec[Y][lb + 1];
                C1[r][lx] = Pc[Y][X];
                C1[r][lb] = Pc[Y][lb + 1];
            }
        }
        __syncthreads();
        const int p2 = t - 2;
        if (p2 >= z0) {
            const float(*Em)[W1] = E1[slot(p2 - 1)];
            const float(*Ec)[W1] = E1[slot(p2)];
            const float(*Ep)[W1] = E1[slot(p2 + 1)];
            const float(*Pm)[W1] = PT1[slot(p2 - 1)];
            const float(*Pc)[W1] = PT1[slot(p2)];
            const float(*Pp)[W1] = PT1[slot(p2 + 1)];
            const float(*Tc)[W1] = TT[slot(p2)];
            const float(*Rc)[W1] = RR[slot(p2)];
            for (int e = tid; e < BH * TY; e += NT) {
                const int r = e / BH, m = e - r * BH;
                const int gy = y0 + r;
                if (gy >= g.n1) continue;
                const int xb = 2 * m + ((gy + p2 + 1) & 1);
                const int xr = 2 * m + ((gy + p2) & 1);
                const int64_t rowoff = g.off0 + (int64_t)gy * g.sy + (int64_t)p2 * g.sz + x0;
                const int X = xb + 1, Y = r + 1;
                if (x0 + xb < g.n0) {
                    NbT<float> ve, vp;
                    LOADNB(ve, Em, Ec, Ep)
                    LOADNB(vp, Pm, Pc, Pp)
#undef LOADNB
                    float Se;
                    const float dq = dq_corr(ve, vp, a.c.a_ih4, Se);
                    const float dQ = dQ_of(dq, Tc[Y][X], a.c);
                    a.eout[rowoff + xb] = (Se - h2 * (dQ + Rc[Y][X] - cb)) * (1.0f / 6.0f);
                }
                if (x0 + xr < g.n0) a.eout[rowoff + xr] = Ec[Y][xr + 1];
            }
        }
        if (pf2) {
            store2(&E0[slot(t + 1)][0][0], ne);
            store2(&PT2[slot(t + 1)][0][0], np);
        }
        if (pf1) {
            store1(&TT[slot(t)][0][0], nt);
            store1(&RR[slot(t)][0][0], nr);
        }
        __syncthreads();
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
__global__ void __launch_bounds__(NT) k_coarse_corr(Geom g, CoefF c, float* e, const float* pt,
                                                    const float* t0, const float* r, int sweeps) {
    constexpr int CM = 1000;
    __shared__ float se[CM], sp[CM], st[CM], sr[CM];
    __shared__ double red[NT / 64];
    const int tid = threadIdx.x;
    for (int64_t q = tid; q < g.nstore; q += NT) {
        se[q] = e[q];
        sp[q] = pt[q];
        st[q] = t0[q];
        sr[q] = r[q];
    }
    __syncthreads();
    const float h2 = c.h2;
    double sumr = 0.0;
    if (!DIR) {
        double acc = 0.0;
        for (int64_t q = tid; q < g.ncell; q += NT) {
            int i, j, k;
            decode(g, q, i, j, k);
            acc += sr[cell_index(g, i, j, k)];
        }
        acc = wave_sum(acc);
        if ((tid & 63) == 0) red[tid >> 6] = acc;
        __syncthreads();
        for (int w = 0; w < NT / 64; ++w) sumr += red[w];
        __syncthreads();
    }
    const int per = (int)((g.ncell + NT - 1) / NT);
    for (int s = 0; s < sweeps; ++s) {
        float cb = 0.0f;
        if (!DIR) {
            double acc = 0.0;
            for (int64_t q = tid; q < g.ncell; q += NT) {
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
            for (int w = 0; w < NT / 64; ++w) sq += red[w];
            cb = (float)((sumr + sq) / (double)g.ncell);
            __syncthreads();
        }
        for (int colour = 0; colour < 2; ++colour) {
            float nv[2];
            int64_t ni[2] = {-1, -1};
            for (int q = 0; q < per && q < 2; ++q) {
                const int64_t m = tid + (int64_t)q * NT;
                if (m >= g.ncell) continue;
                int i, j, k;
                decode(g, m, i, j, k);
                if (((i + j + k) & 1) != colour) continue;
                NbT<float> ve, vp;
                gather_nb<DIR>(g, se, i, j, k, ve);
                gather_nb<DIR>(g, sp, i, j, k, vp);
                const int64_t li = cell_index(g, i, j, k);
                float Se;
                const float dQ = dQ_of(dq_corr(ve, vp, c.a_ih4, Se), st[li], c);
                nv[q] = (Se - h2 * (dQ + sr[li] - cb)) * (1.0f / 6.0f);
                ni[q] = li;
            }
            __syncthreads();
            for (int q = 0; q < 2; ++q)
                if (ni[q] >= 0) se[ni[q]] = nv[q];
            __syncthreads();
        }
    }
    for (int64_t q = tid; q < g.ncell; q += NT) {
        int i, j, k;
        decode(g, q, i, j, k);
        const int64_t li = cell_index(g, i, j, k);
        e[li] = se[li];
    }
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
// launchers
// ---------------------------------------------------------------------------
template <int TY, int DIR>
static hipError_t corr_launch(const CorrArgs& a, hipStream_t s) {
    const int chunks = (a.g.n2 + a.zc - 1) / a.zc;
    hipLaunchKernelGGL((k_smooth_corr<TY, DIR>), dim3(a.tiles_x * a.tiles_y * chunks), dim3(NT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_smooth_corr(const Geom& g, const CoefF& c, const float* ein, float* eout,
                              const float* pt, const float* t0, const float* r, const LevelScalars* sc,
                              SmoothCfg cfg, hipStream_t s) {
    CorrArgs a;
    a.g = g; a.c = c; a.ein = ein; a.eout = eout; a.pt = pt; a.t0 = t0; a.r = r; a.sc = sc;
    a.zc = cfg.zc > 0 ? cfg.zc : 16;
    a.tiles_x = (g.n0 + TX - 1) / TX;
    a.tiles_y = (g.n1 + cfg.ty - 1) / cfg.ty;
    if (g.dir) {
        if (cfg.ty == 4) return corr_launch<4, 1>(a, s);
        if (cfg.ty == 16) return corr_launch<16, 1>(a, s);
        return corr_launch<8, 1>(a, s);
    }
    if (cfg.ty == 4) return corr_launch<4, 0>(a, s);
    if (cfg.ty == 16) return corr_launch<16, 0>(a, s);
    return corr_launch<8, 0>(a, s);
}

hipError_t launch_rr_corr(const Geom& gf, const Geom& gc, const CoefF& c, const float* e, const float* pt,
                          const float* t0, const float* r, const LevelScalars* sc, float* ec, float* eold_c,
                          float* rd_c, double* partials, int* nblocks_out, hipStream_t s) {
    const int nb = grid_for(gc.ncell, 2048);
    if (gf.dir)
        hipLaunchKernelGGL(k_rr_corr<1>, dim3(nb), dim3(NT), 0, s, gf, gc, c, e, pt, t0, r, sc, ec, eold_c, rd_c,
                           partials);
    else
        hipLaunchKernelGGL(k_rr_corr<0>, dim3(nb), dim3(NT), 0, s, gf, gc, c, e, pt, t0, r, sc, ec, eold_c, rd_c,
                           partials);
    *nblocks_out = nb;
    return hipGetLastError();
}

hipError_t launch_fas_corr(const Geom& g, const CoefF& c, const float* e, const float* pt, const float* t0,
                           const float* rd, float* r, double* partials, int* nblocks_out, hipStream_t s) {
    const int nb = grid_for(g.ncell, 2048);
    if (g.dir)
        hipLaunchKernelGGL(k_fas_corr<1>, dim3(nb), dim3(NT), 0, s, g, c, e, pt, t0, rd, r, partials);
    else
        hipLaunchKernelGGL(k_fas_corr<0>, dim3(nb), dim3(NT), 0, s, g, c, e, pt, t0, rd, r, partials);
    *nblocks_out = nb;
    return hipGetLastError();
}

hipError_t launch_prolong_corr(const Geom& gf, const Geom& gc, float* ef, const float* ec, const float* eold_c,
                               hipStream_t s) {
    if (gf.dir)
        hipLaunchKernelGGL(k_prolong_corr<1>, dim3(grid_for(gf.ncell)), dim3(NT), 0, s, gf, gc, ef, ec, eold_c);
    else
        hipLaunchKernelGGL(k_prolong_corr<0>, dim3(grid_for(gf.ncell)), dim3(NT), 0, s, gf, gc, ef, ec, eold_c);
    return hipGetLastError();
}

hipError_t launch_coarse_corr(const Geom& g, const CoefF& c, float* e, const float* pt, const float* t0,
                              const float* r, int sweeps, hipStream_t s) {
    if (g.nstore > 1000 || g.ncell > 2 * NT) return hipErrorInvalidValue;
    if (g.dir)
        hipLaunchKernelGGL(k_coarse_corr<1>, dim3(1), dim3(NT), 0, s, g, c, e, pt, t0, r, sweeps);
    else
        hipLaunchKernelGGL(k_coarse_corr<0>, dim3(1), dim3(NT), 0, s, g, c, e, pt, t0, r, sweeps);
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

}  // namespace vmg
