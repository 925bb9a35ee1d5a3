// gfx950 kernels of the FP64 nonlinear multigrid path.
//
// Discrete operator (Li, Zhao & Koyama, Sec. III.B with w = 1/3, Eq. one_branch):
//   s_x = phi(i+1)+phi(i-1) (likewise y, z), S = s_x+s_y+s_z
//   B_xy = phi(+,+)+phi(-,-)-phi(+,-)-phi(-,+) (likewise xz, yz)
//   Sigma0 h^4 = ((s_x-s_y)^2+(s_x-s_z)^2+(s_y-s_z)^2)/3 + (B_xy^2+B_xz^2+B_yz^2)/8
//   q = alpha*Sigma0 + kappa*delta, D = 1 + (8 alpha/3) q
//   Q = 2q/(1+sqrt D) if D >= 0 else -3/(4 alpha)
//   L(phi) = (S - 6 phi_c)/h^2 - Q
// Sigma0 does not involve phi_c, so the Newton-Gauss-Seidel step of Sec. III.B is
// the exact per-cell root: phi_c <- (S - h^2 (Q + f - cbar)) / 6.
#include <algorithm>
#include <cstring>
#include <type_traits>

#include "brick.h"

namespace vmg {

// ---------------------------------------------------------------------------
// FP64 fused red-black sweep (the z-marching brick is in brick.h).
// ---------------------------------------------------------------------------
struct SmoothArgs {
    Geom g;
    Coef c;
    const double* pin;
    double* pout;
    const double* delta;
    const double* f;      // may be null
    const LevelScalars* sc;
    // prolongation folded into the sweep (periodic): pin += P(uc - oc) first
    Geom gc;
    const double* uc;     // null: no prolongation
    const double* oc;
    int zc, tiles_x, tiles_y;
    // Dirichlet bricks below the finest level: reference of the ghost refresh
    // (null: the ghost shell of pout is left to a separate refresh)
    const double* gref;
};

// FP64 smoother policy of the fused sweep: cells hold phi, sources are delta
// and (on coarse levels) the FAS right-hand side f.  Closed-form update of
// Sec. III.B at w = 1/3: phi_c <- (S - h^2 (Q + f - cbar)) / 6.
template <bool HAS_F>
struct SmoothK {
    using Cell = double;
    using Corr = double;
    // loads two plane steps ahead on the finest level (measured faster); one on
    // coarse levels, whose extra source f would otherwise spill at tile height 8
    static constexpr int AHEAD = HAS_F ? 1 : 2;
    struct Src {
        double dl, f;
    };
    const double* __restrict__ pin;
    double* __restrict__ pout;
    const double* __restrict__ delta;
    const double* __restrict__ f;
    Coef c;
    double inv_h4, h2_6, cb_6;   // 1/h^4, h^2/6, h^2 cbar/6
    float kk;                    // kink_k(h^2)
    Geom gc;                     // folded prolongation: coarse level and its phi^H, phi^H_old
    const double* __restrict__ uc;
    const double* __restrict__ oc;
    const double* __restrict__ gref;

    __device__ SmoothK(const SmoothArgs& a, const Geom& g, bool periodic)
        : pin(a.pin), pout(a.pout), delta(a.delta), f(a.f), c(a.c), gc(a.gc), uc(a.uc), oc(a.oc), gref(a.gref) {
        const double h2 = g.h * g.h;
        inv_h4 = 1.0 / (h2 * h2);
        h2_6 = h2 * (1.0 / 6.0);
        kk = kink_k(h2);
        cb_6 = periodic ? h2_6 * a.sc->cbar : 0.0;
    }
    static constexpr int EB = 8;
    struct InPlane {
        __amdgpu_buffer_rsrc_t u;
    };
    struct SrcPlane {
        __amdgpu_buffer_rsrc_t d, f;
    };
    struct OutPlane {
        __amdgpu_buffer_rsrc_t u;
    };
    __device__ InPlane in_plane(int64_t zo, bool ok) const { return InPlane{plane_rsrc(pin, zo, EB, ok)}; }
    __device__ SrcPlane src_plane(int64_t zo, bool ok) const {
        return SrcPlane{plane_rsrc(delta, zo, EB, ok), plane_rsrc(HAS_F ? f : delta, zo, EB, ok && HAS_F)};
    }
    __device__ OutPlane out_plane(int64_t zo, bool ok) const { return OutPlane{plane_rsrc(pout, zo, EB, ok)}; }
    __device__ double cell_b(const InPlane& P, int bo) const { return buf_ld_f64(P.u, bo); }
    __device__ Src src_b(const SrcPlane& S, int bo) const {
        Src s;
        s.dl = buf_ld_f64(S.d, bo);
        s.f = HAS_F ? buf_ld_f64(S.f, bo) : 0.0;
        return s;
    }
    __device__ void out_b(const OutPlane& O, int bo, double v) const { buf_st_f64(O.u, bo, v); }
    struct CoarsePlane {
        __amdgpu_buffer_rsrc_t u, o;
    };
    __device__ CoarsePlane coarse_plane(int64_t zo) const {
        return CoarsePlane{plane_rsrc(uc, zo, EB, true), plane_rsrc(oc, zo, EB, true)};
    }
    __device__ double coarse_b(const CoarsePlane& C, int bo) const {
        return buf_ld_f64(C.u, bo) - buf_ld_f64(C.o, bo);
    }
    __device__ double add_corr(double u, double v) const { return u + v; }
    __device__ double update_nb(const Nb& v, double centre, const Src& s) const {
        double S, D;
        const double Q = nl_root_d(v, s.dl, c, inv_h4, S, D);
        // (S - h^2 (Q + f - cbar)) / 6, under-relaxed at kink cells
        const double base = HAS_F ? fma(-h2_6, s.f, cb_6) : cb_6;
        return kink_relax(centre, fma(S, 1.0 / 6.0, fma(-h2_6, Q, base)), D, kk);
    }
    // the march reads the centre from LDS only for a kink cell (kink_relax_at)
    template <int W>
    __device__ double update(const double* Pm, const double* Pc, const double* Pp, int co, int o,
                             const Src& s) const {
        Nb v;
        nb_split<W>(Pm, Pc, Pp, co, o, v);
        double S, D;
        const double Q = nl_root_d(v, s.dl, c, inv_h4, S, D);
        const double base = HAS_F ? fma(-h2_6, s.f, cb_6) : cb_6;
        return kink_relax_at(Pc + o, fma(S, 1.0 / 6.0, fma(-h2_6, Q, base)), D, kk);
    }
    // element access of the multi-sweep brick (brick_sweeps)
    __device__ double load_cell(int64_t i) const { return pin[i]; }
    __device__ Src load_src(int64_t i) const {
        Src s;
        s.dl = delta[i];
        s.f = HAS_F ? f[i] : 0.0;
        return s;
    }
    __device__ void store_cell(int64_t i, double v) const { pout[i] = v; }
    __device__ double load_corr(int64_t i) const { return uc[i] - oc[i]; }
    // ghost gi mirrored at interior element ii (sign s) after that cell became v
    __device__ void store_ghost(int64_t gi, int64_t ii, int s, double v) const {
        pout[gi] = gref[gi] + (double)s * (v - gref[ii]);
    }
};

// PRO: the sweep starts from pin + P(uc - oc), the coarse correction prolonged
// as the planes are staged (periodic grids, even z chunks)
template <int TY, int DIR, bool HAS_F, bool DEFER, bool PRO = false>
__global__ void __launch_bounds__(sweep_threads(TY), sweep_waves(TY, DEFER, PRO)) k_smooth(SmoothArgs a) {
    int b = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = b % a.tiles_x;
    b /= a.tiles_x;
    const int ty = b % a.tiles_y;
    const int ch = b / a.tiles_y;
    const int z0 = ch * a.zc;
    if (z0 >= a.g.n2) return;
    const SmoothK<HAS_F> k(a, a.g, DIR == 0);
    fused_sweep<TY, DIR, sweep_threads(TY), DEFER, PRO>(k, a.g, tx * TX, ty * TY, z0, min(z0 + a.zc, a.g.n2));
}

// Persistent sweep over a (grid, tile x, tile y, z chunk) work list: every
// Dirichlet grid of a batch at one level in one launch.  `proto` carries the
// pooled level buffers and coefficients; geoms[w.x] locates grid w.x in them.

// S sweeps (1 or 2) of a small periodic level with a FAS source, one BB^3 brick
// per block (brick_sweeps); PRO adds the prolonged coarse correction first.  The
// two-sweep prolonging variant keeps one block per CU: at two its registers
// spill (measured slower).
template <int S, bool PRO>
__global__ void __launch_bounds__(BRICK_THREADS, (S == 2 && PRO) ? 2 : BRICK_WAVES) k_smooth_brick(SmoothArgs a) {
    const int nbx = (a.g.n0 + BB - 1) / BB, nby = (a.g.n1 + BB - 1) / BB;
    int b = xcd_remap(blockIdx.x, gridDim.x);
    const int bx = b % nbx;
    b /= nbx;
    const int by = b % nby, bz = b / nby;
    const SmoothK<true> k(a, a.g, true);
    brick_sweeps<S, PRO>(k, a.g, bx * BB, by * BB, bz * BB);
}

// One sweep of every Dirichlet grid of a batch at one level on BB^3 bricks:
// items[it] = (grid, brick x, brick y, brick z) of a persistent work list; the
// ghost shell is the boundary (brick_sweeps, DIR = 1).
template <bool HAS_F, bool GHOSTS>
__global__ void __launch_bounds__(BRICK_THREADS, BRICK_WAVES) k_smooth_brick_batch(SmoothArgs proto,
                                                                                   const Geom* __restrict__ geoms,
                                                                                   const int4* __restrict__ items,
                                                                                   int nitems) {
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int4 w = items[it];
        SmoothArgs a = proto;
        a.g = geoms[w.x];
        const SmoothK<HAS_F> k(a, a.g, false);
        brick_sweeps<1, false, 1, GHOSTS>(k, a.g, w.y * BB, w.z * BB, w.w * BB);
        __syncthreads();   // the next item's staging overwrites the LDS
    }
}

template <int TY, bool HAS_F, bool DEFER>
__global__ void __launch_bounds__(sweep_threads(TY), sweep_waves(TY, DEFER)) k_smooth_batch(SmoothArgs proto, const Geom* __restrict__ geoms,
                                                     const int4* __restrict__ items, int nitems) {
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int4 w = items[it];
        SmoothArgs a = proto;
        a.g = geoms[w.x];
        const int z0 = w.w * a.zc;
        const SmoothK<HAS_F> k(a, a.g, false);
        fused_sweep<TY, 1, sweep_threads(TY), DEFER>(k, a.g, w.y * TX, w.z * TY, z0, min(z0 + a.zc, a.g.n2));
    }
}

// residual d = L(phi) + cbar - f at one cell; also returns Q and the guard flag
// ---------------------------------------------------------------------------
// Tiled residual pass.  A block owns a 64 x 8 x zc brick (zc even) and marches
// up z with phi staged on a one-cell ring in LDS (3 planes, next plane
// prefetched into registers).  Thread (m, r) handles the x pair (2m, 2m+1) of
// row r; rows 2k and 2k+1 live in the two halves of one wave, so the 2x2x2
// restriction sums need one cross-half shuffle and one z-pair register.
//   MODE 0 (norm):     d = L(phi) + cbar - f, reductions, optional d_out (caller layout)
//   MODE 1 (restrict): as 0, and R phi -> phic, phiold_c; R d -> rd_c
//   MODE 2 (FAS rhs):  fout = L(phi) - rd (rd passed as f), reductions of Q and fout
// ---------------------------------------------------------------------------
struct ResidArgs {
    Geom g, gc;
    Coef c;
    const double* phi;
    const double* delta;
    const double* f;          // f (modes 0,1) or R d (mode 2); may be null in modes 0,1
    const LevelScalars* sc;
    double* d_out;            // mode 0, optional
    double* phic;             // mode 1
    double* phiold_c;         // mode 1
    double* rd_c;             // mode 1
    double* fout;             // mode 2
    const double* f_fine;     // mode 2, optional: the finer level's f, for tau (R f^h)
    Geom gfine;               // mode 2: geometry of that finer level
    double* partials;
    int zc, tiles_x, tiles_y;
};

constexpr int RTY = 8;   // rows per residual tile

template <int DIR, int MODE>
__global__ void __launch_bounds__(NT) k_resid_tiled(ResidArgs a) {
    constexpr int W1 = TX + 2, H1 = RTY + 2;
    constexpr int NP1 = W1 * H1;
    constexpr int NL1 = (NP1 + NT - 1) / NT;
    __shared__ double PH[3][H1][W1];
    const Geom& g = a.g;
    const int tid = threadIdx.x;
    int b = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = b % a.tiles_x;
    b /= a.tiles_x;
    const int ty = b % a.tiles_y;
    const int ch = b / a.tiles_y;
    const int x0 = tx * TX, y0 = ty * RTY, z0 = ch * a.zc;
    const int z1 = min(z0 + a.zc, g.n2);
    double acc[R_NSLOT] = {0, 0, 0, 0, 0, 0, 0};
    const double cb = (DIR || MODE == 2) ? 0.0 : a.sc->cbar;
    const double inv_h2 = 1.0 / (g.h * g.h), inv_h4 = inv_h2 * inv_h2;
    const int m = tid & 31, r = tid >> 5;           // x pair, row
    const int gy = y0 + r;
    const int xa = x0 + 2 * m;                       // first cell of the pair
    const bool row_ok = gy < g.n1;

    int off1[NL1], lds1[NL1];   // global in-plane offset, LDS word (rows split by parity)
    bool ok1[NL1];
#pragma unroll
    for (int s = 0; s < NL1; ++s) {
        const int e = tid + s * NT;
        ok1[s] = false;
        off1[s] = 0;
        lds1[s] = (e / W1) * W1 + split_col<W1>(e % W1);
        if (e < NP1) {
            int gx = x0 - 1 + e % W1, gyy = y0 - 1 + e / W1;
            if (DIR) {
                ok1[s] = gx >= -1 && gx <= g.n0 && gyy >= -1 && gyy <= g.n1;
            } else {
                gx = wrapi(gx, g.n0);
                gyy = wrapi(gyy, g.n1);
                ok1[s] = true;
            }
            off1[s] = (int)(g.off0 + gx + (int64_t)gyy * g.sy);
        }
    }
    auto plane_off = [&](int t, bool& zok) -> int64_t {
        int gz;
        if (DIR) { gz = t; zok = t >= -1 && t <= g.n2; }
        else { gz = wrapi(t, g.n2); zok = true; }
        return (int64_t)gz * g.sz;
    };
    auto load_plane = [&](int t, double (&rr)[NL1]) {
        bool zok;
        const int64_t zo = plane_off(t, zok);
#pragma unroll
        for (int s = 0; s < NL1; ++s) rr[s] = (ok1[s] && zok && tid + s * NT < NP1) ? a.phi[zo + off1[s]] : 0.0;
    };
    auto store_plane = [&](int sl, const double (&rr)[NL1]) {
        double* dst = &PH[sl][0][0];
#pragma unroll
        for (int s = 0; s < NL1; ++s)
            if (tid + s * NT < NP1) dst[lds1[s]] = rr[s];
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
    double zsum_phi = 0.0, zsum_d = 0.0;   // restriction partial sums of the even plane
    for (int t = z0; t < z1; ++t) {
        // planes t-1, t, t+1 are in LDS; plane t+2 is fetched while plane t is computed
        double nxt[NL1], ndl[2], nfv[2];
        const bool pf = t + 2 <= z1;
        if (pf) load_plane(t + 2, nxt);
        src_fetch(t + 1, ndl, nfv);
        const int sm = slot(t - 1), sc = slot(t), sp = slot(t + 1);
        double psum = 0.0, dsum = 0.0;
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
            const double Q = nl_root(v, cdl[c2], a.c, inv_h4, S, gd);
            const double L = (S - 6.0 * pc) * inv_h2 - Q;
            if (MODE == 2) {
                const double fh = L - cfv[c2];
                a.fout[g.off0 + xa + c2 + (int64_t)gy * g.sy + (int64_t)t * g.sz] = fh;
                acc[R_Q] += Q;
                acc[R_F] += fh;
                // tau^h = L^H(R phi) - R L^h(phi) = f^H - R f^h + cbar^h (a constant on
                // periodic grids): its sums give the RMS of tau^h (Sec. III.C)
                double tau = fh;
                if (a.f_fine) {
                    const Geom& gf = a.gfine;
                    double rf = 0.0;
#pragma unroll
                    for (int m = 0; m < 8; ++m)
                        rf += a.f_fine[cell_index(gf, 2 * (xa + c2) + (m & 1), 2 * gy + ((m >> 1) & 1),
                                                  2 * t + (m >> 2))];
                    tau -= 0.125 * rf;
                }
                acc[R_D1] += tau;
                acc[R_D2] += tau * tau;
            } else {
                const double d = L - cfv[c2] + cb;
                acc[R_D2] += d * d;
                acc[R_D1] += d;
                acc[R_Q] += Q;
                acc[R_F] += cfv[c2];
                acc[R_PHI] += pc;
                acc[R_GUARD] += gd ? 1.0 : 0.0;
                acc[R_NONFIN] += isfinite(d) ? 0.0 : 1.0;
                if (MODE == 0 && a.d_out)
                    a.d_out[xa + c2 + ((int64_t)t * g.n1 + gy) * g.n0] = d;
                psum += pc;
                dsum += d;
            }
        }
        if (MODE == 1) {
            // y pair: rows 2k and 2k+1 are lanes l and l+32 of one wave
            psum += __shfl_down(psum, 32, 64);
            dsum += __shfl_down(dsum, 32, 64);
            if ((t & 1) == 0) {
                zsum_phi = psum;
                zsum_d = dsum;
            } else if ((r & 1) == 0 && row_ok && xa < g.n0) {
                const Geom& gc = a.gc;
                const int64_t co = gc.off0 + (xa >> 1) + (int64_t)(gy >> 1) * gc.sy + (int64_t)(t >> 1) * gc.sz;
                const double rp = 0.125 * (zsum_phi + psum);
                a.phic[co] = rp;
                a.phiold_c[co] = rp;
                a.rd_c[co] = 0.125 * (zsum_d + dsum);
            }
        }
        __syncthreads();
        if (pf) {
            double* dst = &PH[slot(t + 2)][0][0];   // slot of plane t-1: no longer read
#pragma unroll
            for (int s = 0; s < NL1; ++s)
                if (tid + s * NT < NP1) dst[lds1[s]] = nxt[s];
        }
        cdl[0] = ndl[0]; cdl[1] = ndl[1];
        cfv[0] = nfv[0]; cfv[1] = nfv[1];
        __syncthreads();
    }
    block_store_partials(acc, a.partials);
}

static hipError_t resid_launch(ResidArgs& a, int mode, int* nblocks_out, hipStream_t s) {
    a.tiles_x = (a.g.n0 + TX - 1) / TX;
    a.tiles_y = (a.g.n1 + RTY - 1) / RTY;
    a.zc = level_zc((int64_t)a.tiles_x * a.tiles_y, a.g.n2, 32);
    const int nb = a.tiles_x * a.tiles_y * ((a.g.n2 + a.zc - 1) / a.zc);
    *nblocks_out = nb;
#define RL(D, M) hipLaunchKernelGGL((k_resid_tiled<D, M>), dim3(nb), dim3(NT), 0, s, a)
    if (a.g.dir) {
        if (mode == 0) RL(1, 0); else if (mode == 1) RL(1, 1); else RL(1, 2);
    } else {
        if (mode == 0) RL(0, 0); else if (mode == 1) RL(0, 1); else RL(0, 2);
    }
#undef RL
    return hipGetLastError();
}

int resid_blocks(const Geom& g) {
    const int xy = ((g.n0 + TX - 1) / TX) * ((g.n1 + RTY - 1) / RTY);
    const int zc = level_zc(xy, g.n2, 32);
    return xy * ((g.n2 + zc - 1) / zc);
}

// ---------------------------------------------------------------------------
// residual + restriction (8-child average of phi and d) in one pass
// ---------------------------------------------------------------------------
template <int DIR>
__global__ void __launch_bounds__(NT) k_residual_restrict(Geom gf, Geom gc, Coef c,
                                                          const double* __restrict__ phi,
                                                          const double* __restrict__ delta,
                                                          const double* __restrict__ f,
                                                          const LevelScalars* sc, double* phic,
                                                          double* phiold_c, double* rd_c,
                                                          double* partials) {
    double acc[R_NSLOT] = {0, 0, 0, 0, 0, 0, 0};
    const double cb = DIR ? 0.0 : sc->cbar;
    const double inv_h2 = 1.0 / (gf.h * gf.h), inv_h4 = inv_h2 * inv_h2;
    for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < gc.ncell;
         e += (int64_t)gridDim.x * NT) {
        int I, J, K;
        decode(gc, e, I, J, K);
        double sphi = 0.0, sd = 0.0;
#pragma unroll
        for (int ch = 0; ch < 8; ++ch) {
            const int i = 2 * I + (ch & 1), j = 2 * J + ((ch >> 1) & 1), k = 2 * K + (ch >> 2);
            double Q, pc, fv;
            bool gd;
            const double d = cell_residual<DIR>(gf, c, phi, delta, f, cb, i, j, k, inv_h2, inv_h4,
                                                Q, gd, pc, fv);
            acc[R_D2] += d * d;
            acc[R_D1] += d;
            acc[R_Q] += Q;
            acc[R_F] += fv;
            acc[R_PHI] += pc;
            acc[R_GUARD] += gd ? 1.0 : 0.0;
            acc[R_NONFIN] += isfinite(d) ? 0.0 : 1.0;
            sphi += pc;
            sd += d;
        }
        const int64_t co = cell_index(gc, I, J, K);
        phic[co] = 0.125 * sphi;
        phiold_c[co] = 0.125 * sphi;
        rd_c[co] = 0.125 * sd;
    }
    block_store_partials(acc, partials);
}

template <int DIR>
__global__ void __launch_bounds__(NT) k_residual_norm(Geom g, Coef c, const double* __restrict__ phi,
                                                      const double* __restrict__ delta,
                                                      const double* __restrict__ f,
                                                      const LevelScalars* sc, double* d_out,
                                                      double* partials) {
    double acc[R_NSLOT] = {0, 0, 0, 0, 0, 0, 0};
    const double cb = DIR ? 0.0 : sc->cbar;
    const double inv_h2 = 1.0 / (g.h * g.h), inv_h4 = inv_h2 * inv_h2;
    for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < g.ncell;
         e += (int64_t)gridDim.x * NT) {
        int i, j, k;
        decode(g, e, i, j, k);
        double Q, pc, fv;
        bool gd;
        const double d = cell_residual<DIR>(g, c, phi, delta, f, cb, i, j, k, inv_h2, inv_h4, Q, gd,
                                            pc, fv);
        acc[R_D2] += d * d;
        acc[R_D1] += d;
        acc[R_Q] += Q;
        acc[R_F] += fv;
        acc[R_PHI] += pc;
        acc[R_GUARD] += gd ? 1.0 : 0.0;
        acc[R_NONFIN] += isfinite(d) ? 0.0 : 1.0;
        if (d_out) d_out[e] = d;   // caller layout: unpadded, x fastest
    }
    block_store_partials(acc, partials);
}

// f^H = L^H(R phi) - R d   (coarse FAS right-hand side, Sec. III.C)
template <int DIR>
__global__ void __launch_bounds__(NT) k_fas_rhs(Geom g, Coef c, const double* __restrict__ phi,
                                                const double* __restrict__ delta,
                                                const double* __restrict__ rd, double* f,
                                                double* partials) {
    double acc[R_NSLOT] = {0, 0, 0, 0, 0, 0, 0};
    const double inv_h2 = 1.0 / (g.h * g.h), inv_h4 = inv_h2 * inv_h2;
    for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < g.ncell;
         e += (int64_t)gridDim.x * NT) {
        int i, j, k;
        decode(g, e, i, j, k);
        double Q, pc, fv;
        bool gd;
        const double L = cell_residual<DIR>(g, c, phi, delta, nullptr, 0.0, i, j, k, inv_h2, inv_h4,
                                            Q, gd, pc, fv);
        const int64_t gi = cell_index(g, i, j, k);
        const double fh = L - rd[gi];
        f[gi] = fh;
        acc[R_Q] += Q;
        acc[R_F] += fh;
    }
    block_store_partials(acc, partials);
}

// Block b finalizes job b (one launch can close the restriction pass of level
// l and the coarse right-hand-side pass of level l+1).
__global__ void __launch_bounds__(NT) k_finalize(FinJobs jobs) {
    const FinJob& J = jobs.j[blockIdx.x];
    const double* __restrict__ partials = J.partials;
    const int nblocks = J.nblocks, periodic = J.periodic, mode = J.mode;
    const int64_t ncell = J.ncell;
    LevelScalars* sc = J.sc;
    NormOut* out = J.out;
    LevelScalars* inner = J.inner;
    __shared__ double red[NT / 64][R_NSLOT];
    double acc[R_NSLOT];
#pragma unroll
    for (int k = 0; k < R_NSLOT; ++k) acc[k] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += NT) {
#pragma unroll
        for (int k = 0; k < R_NSLOT; ++k) acc[k] += partials[(int64_t)b * R_NSLOT + k];
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < R_NSLOT; ++k) {
        const double s = wave_sum(acc[k]);
        if (lane == 0) red[w][k] = s;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double tot[R_NSLOT];
    for (int k = 0; k < R_NSLOT; ++k) {
        tot[k] = 0.0;
        for (int q = 0; q < NT / 64; ++q) tot[k] += red[q][k];
    }
    const double N = (double)ncell;
    if (mode == 1) {
        if (periodic) sc->cbar = (tot[R_F] + tot[R_Q]) / N;
        if (out) {   // RMS of tau^h over this (coarse) level, mean removed on periodic grids
            const double m = periodic ? tot[R_D1] / N : 0.0;
            out->tau_rms = sqrt(fmax(tot[R_D2] / N - m * m, 0.0));
        }
        return;
    }
    double d2 = tot[R_D2];
    double cb = 0.0;
    if (periodic) {
        const double old = sc->cbar;
        cb = (tot[R_F] + tot[R_Q]) / N;
        const double del = cb - old;
        d2 = tot[R_D2] + 2.0 * del * tot[R_D1] + N * del * del;
        sc->cbar = cb;
    }
    if (mode == 2 && inner) inner->cbar = periodic ? -tot[R_D1] / N : 0.0;
    if (out) {
        out->rms = sqrt(fmax(d2, 0.0) / N);
        out->cbar = cb;
        out->mean_phi = tot[R_PHI] / N;
        out->n_guard = tot[R_GUARD];
        out->n_nonfinite = tot[R_NONFIN];
        out->sum_q = tot[R_Q];
    }
}

// phi^h += P(phi^H - phiold^H): cell-centred trilinear, weights 3/4 and 1/4 per axis
template <int DIR>
__global__ void __launch_bounds__(NT) k_prolong(Geom gf, Geom gc, double* __restrict__ phif,
                                                const double* __restrict__ phic,
                                                const double* __restrict__ oldc) {
    for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < gf.ncell;
         e += (int64_t)gridDim.x * NT) {
        int i, j, k;
        decode(gf, e, i, j, k);
        const int I = i >> 1, J = j >> 1, K = k >> 1;
        const int si = (i & 1) ? 1 : -1, sj = (j & 1) ? 1 : -1, sk = (k & 1) ? 1 : -1;
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            int ii = I + ((q & 1) ? si : 0), jj = J + ((q & 2) ? sj : 0), kk = K + ((q & 4) ? sk : 0);
            const double w = ((q & 1) ? 0.25 : 0.75) * ((q & 2) ? 0.25 : 0.75) * ((q & 4) ? 0.25 : 0.75);
            double corr;
            if (DIR) {
                if (ii < 0 || ii >= gc.n0 || jj < 0 || jj >= gc.n1 || kk < 0 || kk >= gc.n2) {
                    corr = 0.0;
                } else {
                    const int64_t ci = cell_index(gc, ii, jj, kk);
                    corr = phic[ci] - oldc[ci];
                }
            } else {
                ii = ii < 0 ? ii + gc.n0 : (ii >= gc.n0 ? ii - gc.n0 : ii);
                jj = jj < 0 ? jj + gc.n1 : (jj >= gc.n1 ? jj - gc.n1 : jj);
                kk = kk < 0 ? kk + gc.n2 : (kk >= gc.n2 ? kk - gc.n2 : kk);
                const int64_t ci = cell_index(gc, ii, jj, kk);
                corr = phic[ci] - oldc[ci];
            }
            acc += w * corr;
        }
        phif[cell_index(gf, i, j, k)] += acc;
    }
}

// Tiled prolongation + correction.  A block owns a 64 x 8 x pz fine brick
// (pz <= 16, even); the coarse correction c = phi^H - phiold^H of the
// 34 x 6 x (pz/2+2) coarse cells around it is staged in LDS once (zero outside
// a Dirichlet grid, wrapped on a periodic one), then every fine cell adds its
// trilinear interpolant.
constexpr int PZ = 16;   // largest number of fine planes per prolongation block
template <int DIR>
__global__ void __launch_bounds__(NT) k_prolong_tiled(Geom gf, Geom gc, double* __restrict__ phif,
                                                      const double* __restrict__ phic,
                                                      const double* __restrict__ oldc, int tiles_x, int tiles_y,
                                                      int pz) {
    constexpr int CX = TX / 2 + 2, CY = 8 / 2 + 2, CZM = PZ / 2 + 2;
    __shared__ double C[CZM][CY][CX];
    const int CZ = pz / 2 + 2;
    int b = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = b % tiles_x;
    b /= tiles_x;
    const int ty = b % tiles_y;
    const int ch = b / tiles_y;
    const int x0 = tx * TX, y0 = ty * 8, z0 = ch * pz;
    const int cx0 = x0 / 2 - 1, cy0 = y0 / 2 - 1, cz0 = z0 / 2 - 1;
    stage_coarse_diff<DIR>(gc, phic, oldc, C, CZ, cx0, cy0, cz0);
    __syncthreads();
    prolong_tile_rows<4>(gf, phif, C, x0, y0, z0, cx0, cy0, cz0, pz);   // FP64 rows already stream well
}

// ---------------------------------------------------------------------------
// coarsest level: whole grid in LDS, red-black sweeps (same snapshot schedule)
// ---------------------------------------------------------------------------
constexpr int CMAX = 10 * 10 * 10;   // storage of a padded 8^3 grid

// phi (and, if given, phi_also) receive the result; storage starts at g.base.
// With `old` (coarse Dirichlet levels) the ghosts follow the correction phi - old
// by mirroring after every colour pass; without it they stay fixed.
template <int DIR>
__device__ __forceinline__ void coarse_solve_body(Geom g, const Coef& c, double* phi, double* phi_also,
                                                  const double* delta, const double* f, int sweeps,
                                                  const double* old = nullptr) {
    __shared__ double sphi[CMAX], sdel[CMAX], sf[CMAX], sold[CMAX];
    __shared__ double red[NT / 64];
    const int tid = threadIdx.x, nt = blockDim.x;
    phi += g.base;
    delta += g.base;
    if (f) f += g.base;
    if (phi_also) phi_also += g.base;
    if (old) old += g.base;
    for (int64_t e = tid; e < g.nstore; e += nt) {
        sphi[e] = phi[e];
        sdel[e] = delta[e];
        sf[e] = f ? f[e] : 0.0;
        if (DIR && old) sold[e] = old[e];
    }
    __syncthreads();
    Geom lg = g;   // same indexing on the LDS copy
    lg.off0 -= g.base;
    lg.base = 0;
    const int64_t nghost = DIR ? ghost_count_dev(g.n0, g.n1, g.n2) : 0;
    auto refresh_ghosts = [&]() {
        if (!DIR || !old) return;
        for (int64_t q = tid; q < nghost; q += nt) {
            int i, j, k;
            ghost_coords(g.n0, g.n1, g.n2, q, i, j, k);
            int sign = 1;
            const int ir = mirror(i, g.n0, sign), jr = mirror(j, g.n1, sign), kr = mirror(k, g.n2, sign);
            const int64_t gi = cell_index(lg, i, j, k), ii = cell_index(lg, ir, jr, kr);
            sphi[gi] = sold[gi] + sign * (sphi[ii] - sold[ii]);
        }
        __syncthreads();
    };
    const double h2 = g.h * g.h, inv_h4 = 1.0 / (h2 * h2);
    double sumf = 0.0;
    if (!DIR) {
        double a = 0.0;
        for (int64_t e = tid; e < g.ncell; e += nt) {
            int i, j, k;
            decode(g, e, i, j, k);
            a += sf[cell_index(lg, i, j, k)];
        }
        a = wave_sum(a);
        if ((tid & 63) == 0) red[tid >> 6] = a;
        __syncthreads();
        for (int q = 0; q < nt / 64; ++q) sumf += red[q];
        __syncthreads();
    }
    const int per = (int)((g.ncell + nt - 1) / nt);   // <= 2 (checked at launch)
    for (int s = 0; s < sweeps; ++s) {
        double cb = 0.0;
        if (!DIR) {
            double a = 0.0;
            for (int64_t e = tid; e < g.ncell; e += nt) {
                int i, j, k;
                decode(g, e, i, j, k);
                Nb v;
                gather_nb<DIR>(lg, sphi, i, j, k, v);
                double S;
                bool gd;
                a += nl_root(v, sdel[cell_index(lg, i, j, k)], c, inv_h4, S, gd);
            }
            a = wave_sum(a);
            if ((tid & 63) == 0) red[tid >> 6] = a;
            __syncthreads();
            double sq = 0.0;
            for (int q = 0; q < nt / 64; ++q) sq += red[q];
            cb = (sumf + sq) / (double)g.ncell;
            __syncthreads();
        }
        for (int colour = 0; colour < 2; ++colour) {
            double nv[2];
            int64_t ni[2];
            for (int q = 0; q < per && q < 2; ++q) {
                ni[q] = -1;
                const int64_t e = tid + (int64_t)q * nt;
                if (e >= g.ncell) continue;
                int i, j, k;
                decode(g, e, i, j, k);
                if (((i + j + k) & 1) != colour) continue;
                Nb v;
                gather_nb<DIR>(lg, sphi, i, j, k, v);
                const int64_t li = cell_index(lg, i, j, k);
                double S, D;
                const double Q = nl_root_d(v, sdel[li], c, inv_h4, S, D);
                nv[q] = kink_relax(sphi[li], (S - h2 * (Q + sf[li] - cb)) * (1.0 / 6.0), D, kink_k(h2));
                ni[q] = li;
            }
            __syncthreads();
            for (int q = 0; q < per && q < 2; ++q)
                if (tid + (int64_t)q * nt < g.ncell && ni[q] >= 0) sphi[ni[q]] = nv[q];
            __syncthreads();
            refresh_ghosts();
        }
    }
    for (int64_t e = tid; e < g.ncell; e += nt) {
        int i, j, k;
        decode(g, e, i, j, k);
        const int64_t li = cell_index(lg, i, j, k);
        phi[li] = sphi[li];
        if (phi_also) phi_also[li] = sphi[li];
    }
    if (DIR && old)
        for (int64_t q = tid; q < nghost; q += nt) {
            int i, j, k;
            ghost_coords(g.n0, g.n1, g.n2, q, i, j, k);
            const int64_t li = cell_index(lg, i, j, k);
            phi[li] = sphi[li];
            if (phi_also) phi_also[li] = sphi[li];
        }
    __syncthreads();
}

template <int DIR>
__global__ void __launch_bounds__(NT) k_coarse_solve(Geom g, Coef c, double* phi, const double* delta,
                                                     const double* f, int sweeps) {
    coarse_solve_body<DIR>(g, c, phi, nullptr, delta, f, sweeps);
}

// ---------------------------------------------------------------------------
// utilities
// ---------------------------------------------------------------------------
__global__ void k_restrict_plain(Geom gf, Geom gc, const double* uf, double* uc) {
    for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < gc.ncell;
         e += (int64_t)gridDim.x * NT) {
        int I, J, K;
        decode(gc, e, I, J, K);
        double s = 0.0;
        for (int ch = 0; ch < 8; ++ch)
            s += uf[cell_index(gf, 2 * I + (ch & 1), 2 * J + ((ch >> 1) & 1), 2 * K + (ch >> 2))];
        uc[cell_index(gc, I, J, K)] = 0.125 * s;
    }
}

// coarse Dirichlet ghosts: mean of the fine ghost cells inside each coarse ghost cell
__global__ void k_restrict_ghosts(Geom gf, Geom gc, const double* uf, double* uc) {
    const int64_t tot = (int64_t)(gc.n0 + 2) * (gc.n1 + 2) * (gc.n2 + 2);
    for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < tot; e += (int64_t)gridDim.x * NT) {
        const int I = (int)(e % (gc.n0 + 2)) - 1;
        const int J = (int)((e / (gc.n0 + 2)) % (gc.n1 + 2)) - 1;
        const int K = (int)(e / ((int64_t)(gc.n0 + 2) * (gc.n1 + 2))) - 1;
        const int out = (I < 0 || I >= gc.n0) + (J < 0 || J >= gc.n1) + (K < 0 || K >= gc.n2);
        if (out == 0 || out == 3) continue;
        double s = 0.0;
        int cnt = 0;
        for (int ch = 0; ch < 8; ++ch) {
            const int i = 2 * I + (ch & 1), j = 2 * J + ((ch >> 1) & 1), k = 2 * K + (ch >> 2);
            if (i < -1 || i > gf.n0 || j < -1 || j > gf.n1 || k < -1 || k > gf.n2) continue;
            const int o = (i < 0 || i >= gf.n0) + (j < 0 || j >= gf.n1) + (k < 0 || k >= gf.n2);
            if (o == 0 || o == 3) continue;
            s += uf[cell_index(gf, i, j, k)];
            ++cnt;
        }
        uc[cell_index(gc, I, J, K)] = cnt ? s / cnt : 0.0;
    }
}

__global__ void k_copy_in(Geom g, const double* src, double* dst) {
    for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < g.ncell; e += (int64_t)gridDim.x * NT) {
        int i, j, k;
        decode(g, e, i, j, k);
        dst[cell_index(g, i, j, k)] = src[e];
    }
}

__global__ void k_copy_out(Geom g, const double* src, double* dst) {
    for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < g.ncell; e += (int64_t)gridDim.x * NT) {
        int i, j, k;
        decode(g, e, i, j, k);
        dst[e] = src[cell_index(g, i, j, k)];
    }
}

__global__ void k_ghost_in(Geom g, const double* ghost, double* dst, int64_t count) {
    for (int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x; q < count; q += (int64_t)gridDim.x * NT) {
        int i, j, k;
        ghost_coords(g.n0, g.n1, g.n2, q, i, j, k);
        dst[cell_index(g, i, j, k)] = ghost[q];
    }
}

// Trilinear value of a cell-centred periodic parent (np cells of size H) at the
// centre of patch cell c (cells of size h, cell 0 at o*h).
__device__ double parent_trilinear(const double* __restrict__ parent, const int np[3], double H, double h,
                                   const int o[3], const int c[3]) {
    int base[3];
    double t[3];
    for (int d = 0; d < 3; ++d) {
        const double u = (o[d] + c[d] + 0.5) * h / H - 0.5;   // parent index space
        const double fl = floor(u);
        base[d] = (int)fl;
        t[d] = u - fl;
    }
    double v = 0.0;
    for (int m = 0; m < 8; ++m) {
        const int dx = m & 1, dy = (m >> 1) & 1, dz = m >> 2;
        const double w = (dx ? t[0] : 1.0 - t[0]) * (dy ? t[1] : 1.0 - t[1]) * (dz ? t[2] : 1.0 - t[2]);
        const int I = ((base[0] + dx) % np[0] + np[0]) % np[0];
        const int J = ((base[1] + dy) % np[1] + np[1]) % np[1];
        const int K = ((base[2] + dz) % np[2] + np[2]) % np[2];
        v += w * parent[((int64_t)K * np[1] + J) * np[0] + I];
    }
    return v;
}

// MODE 0: ghost shell (compact order); MODE 1: interior, x fastest.
template <int MODE>
__global__ void k_parent_fill(const double* parent, int np0, int np1, int np2, double H, int n0, int n1, int n2,
                              double h, int o0, int o1, int o2, double* out, int64_t count) {
    const int o[3] = {o0, o1, o2}, np[3] = {np0, np1, np2};
    for (int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x; q < count; q += (int64_t)gridDim.x * NT) {
        int c[3];
        if (MODE == 0) {
            ghost_coords(n0, n1, n2, q, c[0], c[1], c[2]);
        } else {
            c[0] = (int)(q % n0);
            c[1] = (int)((q / n0) % n1);
            c[2] = (int)(q / ((int64_t)n0 * n1));
        }
        out[q] = parent_trilinear(parent, np, H, h, o, c);
    }
}

__global__ void k_gauge(Geom g, double* phi, const NormOut* no) {
    const double m = no->mean_phi;
    for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < g.ncell; e += (int64_t)gridDim.x * NT) {
        int i, j, k;
        decode(g, e, i, j, k);
        phi[cell_index(g, i, j, k)] -= m;
    }
}

__global__ void k_fill(double* p, int64_t n, double v) {
    for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT) p[e] = v;
}

__global__ void __launch_bounds__(NT) k_check_finite(const double* p, int64_t n, double* partials) {
    double acc[R_NSLOT] = {0, 0, 0, 0, 0, 0, 0};
    for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT)
        acc[R_NONFIN] += isfinite(p[e]) ? 0.0 : 1.0;
    block_store_partials(acc, partials);
}

// ---------------------------------------------------------------------------
// Batched Dirichlet kernels: one launch covers every grid of a level.  The
// grids of a level share pooled buffers; geoms[k] locates grid k in them and
// each block handles items[blockIdx.x] = (k, first cell) = 256 cells of grid k.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(NT) k_rr_batch(const Geom* __restrict__ gfs, const Geom* __restrict__ gcs,
                                                 const int2* __restrict__ items, Coef c,
                                                 const double* __restrict__ phi, const double* __restrict__ delta,
                                                 const double* __restrict__ f, double* phic, double* phiold_c,
                                                 double* rd_c) {
    // one thread per coarse cell: the children's stencils come out of one 4^3 box;
    // the coarse ghost shell of phic is refreshed here too
    const int2 w = items[blockIdx.x];
    const Geom gf = gfs[w.x], gc = gcs[w.x];
    const int64_t e = (int64_t)w.y + threadIdx.x;
    if (e >= gc.ncell) return;
    const double inv_h2 = 1.0 / (gf.h * gf.h), inv_h4 = inv_h2 * inv_h2;
    int I, J, K;
    decode(gc, e, I, J, K);
    double u[4][4][4];
    load_child_box(gf, phi, I, J, K, u);
    double sphi = 0.0, sd = 0.0;
#pragma unroll
    for (int ch = 0; ch < 8; ++ch) {
        const int a = ch & 1, b = (ch >> 1) & 1, z = ch >> 2;
        Nb v;
        const double pc = box_nb(u, a, b, z, v);
        const int64_t gi = cell_index(gf, 2 * I + a, 2 * J + b, 2 * K + z);
        double S;
        bool gd;
        const double Q = nl_root(v, delta[gi], c, inv_h4, S, gd);
        const double fv = f ? f[gi] : 0.0;
        sd += (S - 6.0 * pc) * inv_h2 - Q - fv;
        sphi += pc;
    }
    const int64_t co = cell_index(gc, I, J, K);
    phic[co] = 0.125 * sphi;
    phiold_c[co] = 0.125 * sphi;
    rd_c[co] = 0.125 * sd;
    copy_ghosts_near(gc, phic, phiold_c, I, J, K);
}

__global__ void __launch_bounds__(NT) k_fas_batch(const Geom* __restrict__ gs, const int2* __restrict__ items,
                                                  Coef c, const double* __restrict__ phi,
                                                  const double* __restrict__ delta, const double* __restrict__ rd,
                                                  double* f) {
    const int2 w = items[blockIdx.x];
    const Geom g = gs[w.x];
    const int64_t e = (int64_t)w.y + threadIdx.x;
    if (e >= g.ncell) return;
    const double inv_h2 = 1.0 / (g.h * g.h), inv_h4 = inv_h2 * inv_h2;
    int i, j, k;
    decode(g, e, i, j, k);
    double Q, pc, fv;
    bool gd;
    const double L = cell_residual<1>(g, c, phi, delta, nullptr, 0.0, i, j, k, inv_h2, inv_h4, Q, gd, pc, fv);
    const int64_t gi = cell_index(g, i, j, k);
    f[gi] = L - rd[gi];
}

// Truncation-error estimate on the next coarser level of every grid (Sec. III.C):
// with phi^H = R phi^h and rd = R d^h just formed by k_rr_batch (d^h = L^h phi^h
// - f^h on Dirichlet grids), tau^h = L^H(R phi^h) - R L^h(phi^h) = L^H(phi^H) -
// rd - R f^h.  Block partials of tau and tau^2 (grid k's blocks are contiguous).
__global__ void __launch_bounds__(ITEM_LANES) k_tau_batch(const Geom* __restrict__ gs, const Geom* __restrict__ gfs,
                                                          const int2* __restrict__ items, Coef c,
                                                          const double* __restrict__ phi,
                                                          const double* __restrict__ delta,
                                                          const double* __restrict__ rd,
                                                          const double* __restrict__ f_fine, double* partials) {
    double acc[R_NSLOT] = {0, 0, 0, 0, 0, 0, 0};
    const int2 w = items[blockIdx.x];
    const Geom g = gs[w.x];
    const double inv_h2 = 1.0 / (g.h * g.h), inv_h4 = inv_h2 * inv_h2;
#pragma unroll
    for (int m = 0; m < ITEM_CELLS / ITEM_LANES; ++m) {
        const int64_t e = (int64_t)w.y + threadIdx.x + m * ITEM_LANES;
        if (e >= g.ncell) break;
        int I, J, K;
        decode(g, e, I, J, K);
        double Q, pc, fv;
        bool gd;
        const double L = cell_residual<1>(g, c, phi, delta, nullptr, 0.0, I, J, K, inv_h2, inv_h4, Q, gd, pc, fv);
        double tau = L - rd[cell_index(g, I, J, K)];
        if (f_fine) {
            const Geom gf = gfs[w.x];
            double rf = 0.0;
#pragma unroll
            for (int q = 0; q < 8; ++q)
                rf += f_fine[cell_index(gf, 2 * I + (q & 1), 2 * J + ((q >> 1) & 1), 2 * K + (q >> 2))];
            tau -= 0.125 * rf;
        }
        acc[R_D1] += tau;
        acc[R_D2] += tau * tau;
    }
    wave_store_partials(acc, partials);
}

// items: 256-cell blocks of the coarse level; each thread adds the prolonged
// correction to the 8 children of its coarse cell
__global__ void __launch_bounds__(NT) k_prolong_batch(const Geom* __restrict__ gfs, const Geom* __restrict__ gcs,
                                                      const int2* __restrict__ items, double* __restrict__ phif,
                                                      const double* __restrict__ phic,
                                                      const double* __restrict__ oldc) {
    const int2 w = items[blockIdx.x];
    const Geom gf = gfs[w.x], gc = gcs[w.x];
    const int64_t e = (int64_t)w.y + threadIdx.x;
    if (e >= gc.ncell) return;
    int I, J, K;
    decode(gc, e, I, J, K);
    prolong_children(gf, gc, phif, phic, oldc, I, J, K);
}

// residual norm partials per block (grid k's blocks are contiguous)
__global__ void __launch_bounds__(ITEM_LANES) k_norm_batch(const Geom* __restrict__ gs,
                                                           const int2* __restrict__ items, Coef c,
                                                           const double* __restrict__ phi,
                                                           const double* __restrict__ delta,
                                                           const double* __restrict__ f, double* partials) {
    double acc[R_NSLOT] = {0, 0, 0, 0, 0, 0, 0};
    const int2 w = items[blockIdx.x];
    const Geom g = gs[w.x];
    const double inv_h2 = 1.0 / (g.h * g.h), inv_h4 = inv_h2 * inv_h2;
#pragma unroll
    for (int m = 0; m < ITEM_CELLS / ITEM_LANES; ++m) {
        const int64_t e = (int64_t)w.y + threadIdx.x + m * ITEM_LANES;
        if (e >= g.ncell) break;
        int i, j, k;
        decode(g, e, i, j, k);
        double Q, pc, fv;
        bool gd;
        const double d = cell_residual<1>(g, c, phi, delta, f, 0.0, i, j, k, inv_h2, inv_h4, Q, gd, pc, fv);
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

// one block per grid: sum its blocks' partials [first[k], first[k+1]) in a fixed order
// tau = 0: the residual norms of the grids; tau = 1: out[k].tau_rms only, the RMS of
// the estimate (no mean removed: a Dirichlet grid has no free constant)
__global__ void __launch_bounds__(NT) k_finalize_batch(const double* __restrict__ partials,
                                                       const int* __restrict__ first,
                                                       const Geom* __restrict__ gs, NormOut* out, int tau) {
    __shared__ double red[NT / 64][R_NSLOT];
    const int k = blockIdx.x;
    double acc[R_NSLOT];
#pragma unroll
    for (int q = 0; q < R_NSLOT; ++q) acc[q] = 0.0;
    for (int b = first[k] + threadIdx.x; b < first[k + 1]; b += NT)
#pragma unroll
        for (int q = 0; q < R_NSLOT; ++q) acc[q] += partials[(int64_t)b * R_NSLOT + q];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < R_NSLOT; ++q) {
        const double s = wave_sum(acc[q]);
        if (lane == 0) red[wv][q] = s;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double tot[R_NSLOT];
    for (int q = 0; q < R_NSLOT; ++q) {
        tot[q] = 0.0;
        for (int m = 0; m < NT / 64; ++m) tot[q] += red[m][q];
    }
    const double N = (double)gs[k].ncell;
    if (tau) {
        out[k].tau_rms = sqrt(fmax(tot[R_D2], 0.0) / N);
        return;
    }
    out[k].rms = sqrt(fmax(tot[R_D2], 0.0) / N);
    out[k].cbar = 0.0;
    out[k].mean_phi = tot[R_PHI] / N;
    out[k].n_guard = tot[R_GUARD];
    out[k].n_nonfinite = tot[R_NONFIN];
    out[k].sum_q = tot[R_Q];
}

// coarsest levels of several grids, one block per grid; the result goes to both
// ping-pong buffers so that either parity reads it
__global__ void __launch_bounds__(NT) k_coarse_batch(const Geom* __restrict__ gs, Coef c, double* phi0,
                                                     double* phi1, const double* delta, const double* f,
                                                     int sweeps, const double* old) {
    coarse_solve_body<1>(gs[blockIdx.x], c, phi0, phi1, delta, f, sweeps, old);
}

__global__ void k_copy_in_batch(const Geom* __restrict__ gs, const int64_t* __restrict__ uoff,
                                const int2* __restrict__ items, const double* __restrict__ src, double* dst0,
                                double* dst1) {
    const int2 w = items[blockIdx.x];
    const Geom g = gs[w.x];
    const int64_t e = (int64_t)w.y + threadIdx.x;
    if (e >= g.ncell) return;
    int i, j, k;
    decode(g, e, i, j, k);
    const double v = src[uoff[w.x] + e];
    const int64_t gi = cell_index(g, i, j, k);
    dst0[gi] = v;
    if (dst1) dst1[gi] = v;
}

__global__ void k_copy_out_batch(const Geom* __restrict__ gs, const int64_t* __restrict__ uoff,
                                 const int2* __restrict__ items, const double* __restrict__ src, double* dst) {
    const int2 w = items[blockIdx.x];
    const Geom g = gs[w.x];
    const int64_t e = (int64_t)w.y + threadIdx.x;
    if (e >= g.ncell) return;
    int i, j, k;
    decode(g, e, i, j, k);
    dst[uoff[w.x] + e] = src[cell_index(g, i, j, k)];
}

// items here run over each grid's ghost values (compact order)
__global__ void k_ghost_in_batch(const Geom* __restrict__ gs, const int64_t* __restrict__ goff,
                                 const int2* __restrict__ items, const double* __restrict__ ghost, double* dst0,
                                 double* dst1) {
    const int2 w = items[blockIdx.x];
    const Geom g = gs[w.x];
    const int64_t q = (int64_t)w.y + threadIdx.x;
    if (q >= ghost_count_dev(g.n0, g.n1, g.n2)) return;
    int i, j, k;
    ghost_coords(g.n0, g.n1, g.n2, q, i, j, k);
    const double v = ghost[goff[w.x] + q];
    const int64_t gi = cell_index(g, i, j, k);
    dst0[gi] = v;
    dst1[gi] = v;
}

__global__ void k_restrict_plain_batch(const Geom* __restrict__ gfs, const Geom* __restrict__ gcs,
                                       const int2* __restrict__ items, const double* __restrict__ uf, double* uc) {
    const int2 w = items[blockIdx.x];
    const Geom gf = gfs[w.x], gc = gcs[w.x];
    const int64_t e = (int64_t)w.y + threadIdx.x;
    if (e >= gc.ncell) return;
    int I, J, K;
    decode(gc, e, I, J, K);
    double s = 0.0;
    for (int ch = 0; ch < 8; ++ch)
        s += uf[cell_index(gf, 2 * I + (ch & 1), 2 * J + ((ch >> 1) & 1), 2 * K + (ch >> 2))];
    uc[cell_index(gc, I, J, K)] = 0.125 * s;
}

// items run over each coarse grid's padded storage; writes the coarse ghost shell
__global__ void k_restrict_ghosts_batch(const Geom* __restrict__ gfs, const Geom* __restrict__ gcs,
                                        const int2* __restrict__ items, const double* __restrict__ uf,
                                        double* uc0, double* uc1, double* uc2) {
    const int2 w = items[blockIdx.x];
    const Geom gf = gfs[w.x], gc = gcs[w.x];
    const int64_t e = (int64_t)w.y + threadIdx.x;
    if (e >= gc.nstore) return;
    const int I = (int)(e % (gc.n0 + 2)) - 1;
    const int J = (int)((e / (gc.n0 + 2)) % (gc.n1 + 2)) - 1;
    const int K = (int)(e / ((int64_t)(gc.n0 + 2) * (gc.n1 + 2))) - 1;
    const int out = (I < 0 || I >= gc.n0) + (J < 0 || J >= gc.n1) + (K < 0 || K >= gc.n2);
    if (out == 0 || out == 3) return;
    double s = 0.0;
    int cnt = 0;
    for (int ch = 0; ch < 8; ++ch) {
        const int i = 2 * I + (ch & 1), j = 2 * J + ((ch >> 1) & 1), k = 2 * K + (ch >> 2);
        if (i < -1 || i > gf.n0 || j < -1 || j > gf.n1 || k < -1 || k > gf.n2) continue;
        const int o = (i < 0 || i >= gf.n0) + (j < 0 || j >= gf.n1) + (k < 0 || k >= gf.n2);
        if (o == 0 || o == 3) continue;
        s += uf[cell_index(gf, i, j, k)];
        ++cnt;
    }
    const double v = cnt ? s / cnt : 0.0;
    const int64_t ci = cell_index(gc, I, J, K);
    uc0[ci] = v;
    uc1[ci] = v;
    uc2[ci] = v;
}

__global__ void __launch_bounds__(NT) k_check_finite_batch(const Geom* __restrict__ gs,
                                                           const int64_t* __restrict__ uoff,
                                                           const int2* __restrict__ items,
                                                           const double* __restrict__ src, double* partials) {
    double acc[R_NSLOT] = {0, 0, 0, 0, 0, 0, 0};
    const int2 w = items[blockIdx.x];
    const Geom g = gs[w.x];
    const int64_t e = (int64_t)w.y + threadIdx.x;
    if (e < g.ncell) acc[R_NONFIN] = isfinite(src[uoff[w.x] + e]) ? 0.0 : 1.0;
    block_store_partials(acc, partials);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int partial_blocks_for(int64_t ncell) { return grid_for(ncell, MAX_RED_BLOCKS); }

int64_t ghost_count(int n0, int n1, int n2) {
    return 2 * ((int64_t)n1 * n2 + (int64_t)n0 * n2 + (int64_t)n0 * n1) + 4 * ((int64_t)n0 + n1 + n2);
}

template <int TY, int DIR>
static hipError_t smooth_launch(const SmoothArgs& a, bool defer, hipStream_t s) {
    const int chunks = (a.g.n2 + a.zc - 1) / a.zc;
    const int nb = a.tiles_x * a.tiles_y * chunks;
    if (!DIR && a.uc) {
        if (a.f) {
            if (defer) hipLaunchKernelGGL((k_smooth<TY, 0, true, true, true>), dim3(nb), dim3(sweep_threads(TY)), 0, s, a);
            else hipLaunchKernelGGL((k_smooth<TY, 0, true, false, true>), dim3(nb), dim3(sweep_threads(TY)), 0, s, a);
        } else {
            if (defer) hipLaunchKernelGGL((k_smooth<TY, 0, false, true, true>), dim3(nb), dim3(sweep_threads(TY)), 0, s, a);
            else hipLaunchKernelGGL((k_smooth<TY, 0, false, false, true>), dim3(nb), dim3(sweep_threads(TY)), 0, s, a);
        }
        return hipGetLastError();
    }
    if (a.f) {
        if (defer) hipLaunchKernelGGL((k_smooth<TY, DIR, true, true>), dim3(nb), dim3(sweep_threads(TY)), 0, s, a);
        else hipLaunchKernelGGL((k_smooth<TY, DIR, true, false>), dim3(nb), dim3(sweep_threads(TY)), 0, s, a);
    } else {
        if (defer) hipLaunchKernelGGL((k_smooth<TY, DIR, false, true>), dim3(nb), dim3(sweep_threads(TY)), 0, s, a);
        else hipLaunchKernelGGL((k_smooth<TY, DIR, false, false>), dim3(nb), dim3(sweep_threads(TY)), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_smooth(const Geom& g, const Coef& c, const double* pin, double* pout,
                         const double* delta, const double* f, const LevelScalars* sc,
                         SmoothCfg cfg, hipStream_t s, const ProlongIn* pro, int nsweeps) {
    SmoothArgs a;
    std::memset(&a, 0, sizeof(a));
    a.g = g; a.c = c; a.pin = pin; a.pout = pout; a.delta = delta; a.f = f; a.sc = sc;
    if (cfg.pipe == PIPE_BRICK) {
        // periodic coarse levels (with their FAS source), one or two sweeps
        if (g.dir || !f || nsweeps < 1 || nsweeps > 2) return hipErrorInvalidValue;
        if (pro) {
            if (!can_fold_prolong(g, pro->gc, 2)) return hipErrorInvalidValue;
            a.gc = pro->gc;
            a.uc = pro->uc;
            a.oc = pro->oc;
        }
        const dim3 nb(((g.n0 + BB - 1) / BB) * ((g.n1 + BB - 1) / BB) * ((g.n2 + BB - 1) / BB));
        if (nsweeps == 2) {
            if (pro) hipLaunchKernelGGL((k_smooth_brick<2, true>), nb, dim3(BRICK_THREADS), 0, s, a);
            else hipLaunchKernelGGL((k_smooth_brick<2, false>), nb, dim3(BRICK_THREADS), 0, s, a);
        } else {
            if (pro) hipLaunchKernelGGL((k_smooth_brick<1, true>), nb, dim3(BRICK_THREADS), 0, s, a);
            else hipLaunchKernelGGL((k_smooth_brick<1, false>), nb, dim3(BRICK_THREADS), 0, s, a);
        }
        return hipGetLastError();
    }
    if (nsweeps != 1) return hipErrorInvalidValue;
    a.zc = cfg.zc > 0 ? cfg.zc : 16;
    if (pro) {
        if (!can_fold_prolong(g, pro->gc, a.zc)) return hipErrorInvalidValue;
        a.gc = pro->gc;
        a.uc = pro->uc;
        a.oc = pro->oc;
    }
    a.tiles_x = (g.n0 + TX - 1) / TX;
    const int ty = cfg.ty;
    a.tiles_y = (g.n1 + ty - 1) / ty;
    const bool d = cfg.pipe != 0;
    if (g.dir) {
        if (ty == 4) return smooth_launch<4, 1>(a, d, s);
        if (ty == 16) return smooth_launch<16, 1>(a, d, s);
        if (ty == 12) return smooth_launch<12, 1>(a, d, s);
        return smooth_launch<8, 1>(a, d, s);
    }
    if (ty == 4) return smooth_launch<4, 0>(a, d, s);
    if (ty == 16) return smooth_launch<16, 0>(a, d, s);
    if (ty == 12) return smooth_launch<12, 0>(a, d, s);
    return smooth_launch<8, 0>(a, d, s);
}

hipError_t launch_residual_restrict(const Geom& gf, const Geom& gc, const Coef& c,
                                    const double* phi, const double* delta, const double* f,
                                    const LevelScalars* sc, double* phic, double* phiold_c,
                                    double* rd_c, double* partials, int* nblocks_out, hipStream_t s) {
    ResidArgs a;
    std::memset(&a, 0, sizeof(a));
    a.g = gf; a.gc = gc; a.c = c; a.phi = phi; a.delta = delta; a.f = f; a.sc = sc;
    a.phic = phic; a.phiold_c = phiold_c; a.rd_c = rd_c; a.partials = partials;
    return resid_launch(a, 1, nblocks_out, s);
}

hipError_t launch_residual_norm(const Geom& g, const Coef& c, const double* phi,
                                const double* delta, const double* f, const LevelScalars* sc,
                                double* d_out, double* partials, int* nblocks_out, hipStream_t s) {
    ResidArgs a;
    std::memset(&a, 0, sizeof(a));
    a.g = g; a.c = c; a.phi = phi; a.delta = delta; a.f = f; a.sc = sc; a.d_out = d_out;
    a.partials = partials;
    return resid_launch(a, 0, nblocks_out, s);
}

hipError_t launch_fas_rhs(const Geom& g, const Coef& c, const double* phi, const double* delta,
                          const double* rd, double* f, double* partials, int* nblocks_out,
                          hipStream_t s, const double* f_fine, const Geom* gfine) {
    ResidArgs a;
    std::memset(&a, 0, sizeof(a));
    a.g = g; a.c = c; a.phi = phi; a.delta = delta; a.f = rd; a.fout = f; a.partials = partials;
    a.f_fine = f_fine;
    if (gfine) a.gfine = *gfine;
    return resid_launch(a, 2, nblocks_out, s);
}

hipError_t launch_finalize(const double* partials, int nblocks, int64_t ncell, int periodic,
                           int mode, LevelScalars* sc, NormOut* out, hipStream_t s, LevelScalars* inner) {
    FinJobs j;
    j.j[0] = FinJob{partials, nblocks, periodic, mode, ncell, sc, out, inner};
    j.j[1] = j.j[0];
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(NT), 0, s, j);
    return hipGetLastError();
}

hipError_t launch_finalize_pair(const FinJob& a, const FinJob& b, hipStream_t s) {
    FinJobs j;
    j.j[0] = a;
    j.j[1] = b;
    hipLaunchKernelGGL(k_finalize, dim3(2), dim3(NT), 0, s, j);
    return hipGetLastError();
}

hipError_t launch_prolong(const Geom& gf, const Geom& gc, double* phif, const double* phic,
                          const double* phiold_c, hipStream_t s) {
    const int tx = (gf.n0 + TX - 1) / TX, ty = (gf.n1 + 7) / 8;
    const int pz = level_zc((int64_t)tx * ty, gf.n2, PZ);
    const int nb = tx * ty * ((gf.n2 + pz - 1) / pz);
    if (gf.dir)
        hipLaunchKernelGGL(k_prolong_tiled<1>, dim3(nb), dim3(NT), 0, s, gf, gc, phif, phic, phiold_c, tx, ty, pz);
    else
        hipLaunchKernelGGL(k_prolong_tiled<0>, dim3(nb), dim3(NT), 0, s, gf, gc, phif, phic, phiold_c, tx, ty, pz);
    return hipGetLastError();
}

hipError_t launch_coarse_solve(const Geom& g, const Coef& c, double* phi, const double* delta,
                               const double* f, LevelScalars* sc, int sweeps, hipStream_t s) {
    (void)sc;
    if (g.nstore > CMAX || g.ncell > 2 * NT) return hipErrorInvalidValue;
    const int nt = g.ncell <= 128 ? 64 : NT;   // one wave for small grids: cheap barriers
    if (g.dir)
        hipLaunchKernelGGL(k_coarse_solve<1>, dim3(1), dim3(nt), 0, s, g, c, phi, delta, f, sweeps);
    else
        hipLaunchKernelGGL(k_coarse_solve<0>, dim3(1), dim3(nt), 0, s, g, c, phi, delta, f, sweeps);
    return hipGetLastError();
}

hipError_t launch_restrict_plain(const Geom& gf, const Geom& gc, const double* uf, double* uc,
                                 hipStream_t s) {
    hipLaunchKernelGGL(k_restrict_plain, dim3(grid_for(gc.ncell)), dim3(NT), 0, s, gf, gc, uf, uc);
    return hipGetLastError();
}

hipError_t launch_restrict_ghosts(const Geom& gf, const Geom& gc, const double* uf, double* uc,
                                  hipStream_t s) {
    const int64_t tot = (int64_t)(gc.n0 + 2) * (gc.n1 + 2) * (gc.n2 + 2);
    hipLaunchKernelGGL(k_restrict_ghosts, dim3(grid_for(tot)), dim3(NT), 0, s, gf, gc, uf, uc);
    return hipGetLastError();
}

hipError_t launch_copy_in(const Geom& g, const double* src, double* dst, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_in, dim3(grid_for(g.ncell)), dim3(NT), 0, s, g, src, dst);
    return hipGetLastError();
}

hipError_t launch_copy_out(const Geom& g, const double* src, double* dst, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_out, dim3(grid_for(g.ncell)), dim3(NT), 0, s, g, src, dst);
    return hipGetLastError();
}

hipError_t launch_ghost_in(const Geom& g, const double* ghost, double* dst, hipStream_t s) {
    const int64_t cnt = ghost_count(g.n0, g.n1, g.n2);
    hipLaunchKernelGGL(k_ghost_in, dim3(grid_for(cnt)), dim3(NT), 0, s, g, ghost, dst, cnt);
    return hipGetLastError();
}

hipError_t launch_ghost_fill(const double* parent, int np0, int np1, int np2, double H, int n0,
                             int n1, int n2, double h, int o0, int o1, int o2, double* ghost,
                             hipStream_t s) {
    const int64_t cnt = ghost_count(n0, n1, n2);
    hipLaunchKernelGGL(k_parent_fill<0>, dim3(grid_for(cnt)), dim3(NT), 0, s, parent, np0, np1, np2, H,
                       n0, n1, n2, h, o0, o1, o2, ghost, cnt);
    return hipGetLastError();
}

// Total potential Psi = phi_N + phi/2 and acceleration -grad Psi (periodic
// central differences).  A block of FX x FY threads owns an FX x FY column of
// cells and marches up a chunk of FZC planes: Psi of each plane, with a
// one-cell ring, is staged in LDS (two buffers: plane k and k + 1), so each
// input is read about once; the z neighbours are the previous plane's value
// (kept in a register) and the next plane's tile.
constexpr int FX = 64, FY = 8, FZC = 16, FNT = FX * FY;
constexpr int FW = FX + 2, FH = FY + 2, FNP = FW * FH, FNL = (FNP + FNT - 1) / FNT;

__global__ void __launch_bounds__(FNT) k_total_force(int n0, int n1, int n2, double inv_2h,
                                                    const double* __restrict__ phin,
                                                    const double* __restrict__ phi, double* __restrict__ psi,
                                                    double* __restrict__ g) {
    __shared__ double T[2][FH][FW];
    const int tiles_x = (n0 + FX - 1) / FX, tiles_y = (n1 + FY - 1) / FY;
    int b = blockIdx.x;
    const int tx = b % tiles_x;
    b /= tiles_x;
    const int ty = b % tiles_y;
    const int z0 = (b / tiles_y) * FZC, z1 = min(z0 + FZC, n2);
    const int lx = threadIdx.x % FX, ly = threadIdx.x / FX;
    const int i = tx * FX + lx, j = ty * FY + ly;
    const bool active = i < n0 && j < n1;
    const int64_t N = (int64_t)n0 * n1 * n2, pl = (int64_t)n0 * n1;
    // in-plane offsets of this thread's loader slots (ring included, periodic wrap)
    int64_t off[FNL];
#pragma unroll
    for (int s2 = 0; s2 < FNL; ++s2) {
        const int e = threadIdx.x + s2 * FNT;
        off[s2] = 0;
        if (e < FNP) {
            int gx = (tx * FX - 1 + e % FW) % n0, gy = (ty * FY - 1 + e / FW) % n1;
            gx += gx < 0 ? n0 : 0;
            gy += gy < 0 ? n1 : 0;
            off[s2] = (int64_t)gy * n0 + gx;
        }
    }
    auto P = [&](int64_t q) { return phin[q] + 0.5 * phi[q]; };
    auto load_tile = [&](int buf, int k) {
        const int64_t zo = (int64_t)k * pl;
#pragma unroll
        for (int s2 = 0; s2 < FNL; ++s2) {
            const int e = threadIdx.x + s2 * FNT;
            if (e < FNP) T[buf][e / FW][e % FW] = P(zo + off[s2]);
        }
    };
    const int64_t col = active ? (int64_t)j * n0 + i : 0;
    double pm = P((int64_t)(z0 == 0 ? n2 - 1 : z0 - 1) * pl + col);     // Psi at (i, j, z0 - 1)
    load_tile(0, z0);
    int cur = 0;
    for (int k = z0; k < z1; ++k) {
        load_tile(cur ^ 1, k + 1 == n2 ? 0 : k + 1);
        __syncthreads();
        const double pc = T[cur][ly + 1][lx + 1];
        const double pp = T[cur ^ 1][ly + 1][lx + 1];
        if (active) {
            const int64_t e = (int64_t)k * pl + col;
            if (psi) psi[e] = pc;
            g[e] = -(T[cur][ly + 1][lx + 2] - T[cur][ly + 1][lx]) * inv_2h;
            g[N + e] = -(T[cur][ly + 2][lx + 1] - T[cur][ly][lx + 1]) * inv_2h;
            g[2 * N + e] = -(pp - pm) * inv_2h;
        }
        pm = pc;
        cur ^= 1;
        __syncthreads();
    }
}

int64_t total_force_blocks(int n0, int n1, int n2) {
    return (int64_t)((n0 + FX - 1) / FX) * ((n1 + FY - 1) / FY) * ((n2 + FZC - 1) / FZC);
}

hipError_t launch_total_force(int n0, int n1, int n2, double h, const double* phin, const double* phi, double* psi,
                              double* g, hipStream_t s) {
    hipLaunchKernelGGL(k_total_force, dim3((unsigned)total_force_blocks(n0, n1, n2)), dim3(FNT), 0, s, n0, n1, n2,
                       1.0 / (2.0 * h), phin, phi, psi, g);
    return hipGetLastError();
}

hipError_t launch_interior_fill(const double* parent, int np0, int np1, int np2, double H, int n0, int n1, int n2,
                                double h, int o0, int o1, int o2, double* phi, hipStream_t s) {
    const int64_t cnt = (int64_t)n0 * n1 * n2;
    hipLaunchKernelGGL(k_parent_fill<1>, dim3(grid_for(cnt)), dim3(NT), 0, s, parent, np0, np1, np2, H,
                       n0, n1, n2, h, o0, o1, o2, phi, cnt);
    return hipGetLastError();
}

hipError_t launch_gauge(const Geom& g, double* phi, const NormOut* no, hipStream_t s) {
    hipLaunchKernelGGL(k_gauge, dim3(grid_for(g.ncell)), dim3(NT), 0, s, g, phi, no);
    return hipGetLastError();
}

hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(NT), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_check_finite(const double* p, int64_t n, double* partials, int* nblocks_out,
                               hipStream_t s) {
    const int nb = grid_for(n, MAX_RED_BLOCKS);
    hipLaunchKernelGGL(k_check_finite, dim3(nb), dim3(NT), 0, s, p, n, partials);
    *nblocks_out = nb;
    return hipGetLastError();
}

// ---- batched launchers --------------------------------------------------------
template <int TY>
static void smooth_batch_ty(const SmoothArgs& proto, const Geom* geoms, const int4* items, int nitems, int nb,
                            bool defer, hipStream_t s) {
    const bool f = proto.f != nullptr;
    if (f && defer) hipLaunchKernelGGL((k_smooth_batch<TY, true, true>), dim3(nb), dim3(sweep_threads(TY)), 0, s, proto, geoms, items, nitems);
    else if (f) hipLaunchKernelGGL((k_smooth_batch<TY, true, false>), dim3(nb), dim3(sweep_threads(TY)), 0, s, proto, geoms, items, nitems);
    else if (defer) hipLaunchKernelGGL((k_smooth_batch<TY, false, true>), dim3(nb), dim3(sweep_threads(TY)), 0, s, proto, geoms, items, nitems);
    else hipLaunchKernelGGL((k_smooth_batch<TY, false, false>), dim3(nb), dim3(sweep_threads(TY)), 0, s, proto, geoms, items, nitems);
}

hipError_t launch_smooth_batch(const SmoothArgs& proto, const Geom* geoms, const int4* items, int nitems,
                               SmoothCfg cfg, int max_blocks, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    const int nb = std::min(nitems, max_blocks);
    if (cfg.pipe == PIPE_BRICK) {
        const dim3 g(nb), t(BRICK_THREADS);
        if (proto.f && proto.gref) hipLaunchKernelGGL((k_smooth_brick_batch<true, true>), g, t, 0, s, proto, geoms, items, nitems);
        else if (proto.f) hipLaunchKernelGGL((k_smooth_brick_batch<true, false>), g, t, 0, s, proto, geoms, items, nitems);
        else if (proto.gref) hipLaunchKernelGGL((k_smooth_brick_batch<false, true>), g, t, 0, s, proto, geoms, items, nitems);
        else hipLaunchKernelGGL((k_smooth_brick_batch<false, false>), g, t, 0, s, proto, geoms, items, nitems);
        return hipGetLastError();
    }
    if (proto.gref) return hipErrorInvalidValue;   // the march leaves the ghosts to a separate refresh
    const bool d = cfg.pipe != 0;
    if (cfg.ty == 4) smooth_batch_ty<4>(proto, geoms, items, nitems, nb, d, s);
    else if (cfg.ty == 16) smooth_batch_ty<16>(proto, geoms, items, nitems, nb, d, s);
    else if (cfg.ty == 12) smooth_batch_ty<12>(proto, geoms, items, nitems, nb, d, s);
    else smooth_batch_ty<8>(proto, geoms, items, nitems, nb, d, s);
    return hipGetLastError();
}

hipError_t launch_smooth_batch_args(const Coef& c, const double* pin, double* pout, const double* delta,
                                    const double* f, SmoothCfg cfg, const Geom* geoms, const int4* items,
                                    int nitems, int max_blocks, hipStream_t s, const double* gref) {
    SmoothArgs a;
    std::memset(&a, 0, sizeof(a));
    a.c = c; a.pin = pin; a.pout = pout; a.delta = delta; a.f = f; a.sc = nullptr; a.gref = gref;
    a.zc = cfg.zc > 0 ? cfg.zc : 16;
    return launch_smooth_batch(a, geoms, items, nitems, cfg, max_blocks, s);
}

hipError_t launch_rr_batch(const Geom* gfs, const Geom* gcs, const int2* items, int nitems, const Coef& c,
                           const double* phi, const double* delta, const double* f, double* phic,
                           double* phiold_c, double* rd_c, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rr_batch, dim3(nitems), dim3(NT), 0, s, gfs, gcs, items, c, phi, delta, f, phic, phiold_c,
                       rd_c);
    return hipGetLastError();
}

hipError_t launch_fas_batch(const Geom* gs, const int2* items, int nitems, const Coef& c, const double* phi,
                            const double* delta, const double* rd, double* f, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fas_batch, dim3(nitems), dim3(NT), 0, s, gs, items, c, phi, delta, rd, f);
    return hipGetLastError();
}

hipError_t launch_tau_batch(const Geom* gs, const Geom* gfs, const int2* items, int nitems, const Coef& c,
                            const double* phi, const double* delta, const double* rd, const double* f_fine,
                            double* partials, const int* first, int ngrids, NormOut* out, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tau_batch, dim3(nitems), dim3(ITEM_LANES), 0, s, gs, gfs, items, c, phi, delta, rd, f_fine,
                       partials);
    hipLaunchKernelGGL(k_finalize_batch, dim3(ngrids), dim3(NT), 0, s, partials, first, gs, out, 1);
    return hipGetLastError();
}

hipError_t launch_prolong_batch(const Geom* gfs, const Geom* gcs, const int2* items, int nitems, double* phif,
                                const double* phic, const double* oldc, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_prolong_batch, dim3(nitems), dim3(NT), 0, s, gfs, gcs, items, phif, phic, oldc);
    return hipGetLastError();
}

hipError_t launch_norm_batch(const Geom* gs, const int2* items, int nitems, const Coef& c, const double* phi,
                             const double* delta, const double* f, double* partials, const int* first, int ngrids,
                             NormOut* out, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_norm_batch, dim3(nitems), dim3(ITEM_LANES), 0, s, gs, items, c, phi, delta, f, partials);
    hipLaunchKernelGGL(k_finalize_batch, dim3(ngrids), dim3(NT), 0, s, partials, first, gs, out, 0);
    return hipGetLastError();
}

hipError_t launch_finalize_batch(const double* partials, const int* first, const Geom* gs, int ngrids,
                                 NormOut* out, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize_batch, dim3(ngrids), dim3(NT), 0, s, partials, first, gs, out, 0);
    return hipGetLastError();
}

hipError_t launch_coarse_batch(const Geom* gs, int ngrids, const Coef& c, double* phi0, double* phi1,
                               const double* delta, const double* f, int sweeps, const double* old,
                               hipStream_t s) {
    if (ngrids <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_coarse_batch, dim3(ngrids), dim3(NT), 0, s, gs, c, phi0, phi1, delta, f, sweeps, old);
    return hipGetLastError();
}

hipError_t launch_ghost_refresh_batch(const Geom* gs, const int2* items, int nitems, double* u, const double* ref,
                                      hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ghost_refresh_batch<double>, dim3(nitems), dim3(NT), 0, s, gs, items, u, ref);
    return hipGetLastError();
}

hipError_t launch_ghost_refresh_batch_f(const Geom* gs, const int2* items, int nitems, float* u, const float* ref,
                                        hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ghost_refresh_batch<float>, dim3(nitems), dim3(NT), 0, s, gs, items, u, ref);
    return hipGetLastError();
}

hipError_t launch_copy_in_batch(const Geom* gs, const int64_t* uoff, const int2* items, int nitems,
                                const double* src, double* dst0, double* dst1, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_in_batch, dim3(nitems), dim3(NT), 0, s, gs, uoff, items, src, dst0, dst1);
    return hipGetLastError();
}

hipError_t launch_copy_out_batch(const Geom* gs, const int64_t* uoff, const int2* items, int nitems,
                                 const double* src, double* dst, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_out_batch, dim3(nitems), dim3(NT), 0, s, gs, uoff, items, src, dst);
    return hipGetLastError();
}

hipError_t launch_ghost_in_batch(const Geom* gs, const int64_t* goff, const int2* items, int nitems,
                                 const double* ghost, double* dst0, double* dst1, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ghost_in_batch, dim3(nitems), dim3(NT), 0, s, gs, goff, items, ghost, dst0, dst1);
    return hipGetLastError();
}

hipError_t launch_restrict_plain_batch(const Geom* gfs, const Geom* gcs, const int2* items, int nitems,
                                       const double* uf, double* uc, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_restrict_plain_batch, dim3(nitems), dim3(NT), 0, s, gfs, gcs, items, uf, uc);
    return hipGetLastError();
}

hipError_t launch_restrict_ghosts_batch(const Geom* gfs, const Geom* gcs, const int2* items, int nitems,
                                        const double* uf, double* uc0, double* uc1, double* uc2, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_restrict_ghosts_batch, dim3(nitems), dim3(NT), 0, s, gfs, gcs, items, uf, uc0, uc1, uc2);
    return hipGetLastError();
}

hipError_t launch_check_finite_batch(const Geom* gs, const int64_t* uoff, const int2* items, int nitems,
                                     const double* src, double* partials, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_finite_batch, dim3(nitems), dim3(NT), 0, s, gs, uoff, items, src, partials);
    return hipGetLastError();
}

}  // namespace vmg
