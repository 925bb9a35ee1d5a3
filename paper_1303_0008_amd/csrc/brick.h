// Fused red-black Gauss-Seidel sweep over one TX x TY x (z1 - z0) brick,
// shared by the FP64 smoother and the FP32 correction smoother.
//
// Colour of cell (i,j,k) = (i+j+k) & 1 (0 = red).  The red phase reads only the
// old state u^0 (so same-colour edge neighbours come from the snapshot); the
// black phase reads u^1 = u^0 with the red cells updated.  A block marches up z:
//   * u^0 is staged in LDS on a two-cell ring around the tile (3 planes),
//   * the red phase runs on a one-cell ring (recomputing what neighbouring
//     blocks own, so no block reads another block's output) and stores the
//     full u^1 plane (red computed, black copied) in LDS (3 planes),
//   * the black phase runs on the tile and writes u^2 once.
// Loads run one or two plane steps ahead of their use (K::AHEAD, see the
// pipeline below); a sweep reads u^0 and the per-cell sources once and writes
// u^2 once.
//
// The arithmetic lives in a policy K:
//   K::Cell                 what a cell holds in LDS (double phi, or float2 (e, phi~))
//   K::Src                  per-cell sources of the update (delta and f, or t0 and r)
//   K::AHEAD                plane steps the loads run ahead of their use (1 or 2)
//   K::EB                   bytes of one element of the policy's arrays
//   k.in_plane(zo, ok), k.src_plane(zo, ok), k.out_plane(zo, ok)
//                           buffer resources of the input state / sources / output
//                           for the plane starting at element zo (ok false: all
//                           accesses out of range, i.e. zero)
//   k.cell_b(P, bo), k.src_b(S, bo)   the input state / sources at byte offset bo
//                           of a plane (out of range: zero)
//   k.template update<W>(Pm, Pc, Pp, c, o, src)   updated cell from its neighbourhood
//   k.out_b(O, bo, cell)    write the output state at byte offset bo (out of range:
//                           dropped)
// and, for a sweep that first adds the prolonged coarse correction (PRO):
//   K::Corr                 type of the coarse correction u^H - u^H_old
//   k.gc                    the coarse level's geometry
//   k.coarse_plane(zo), k.coarse_b(C, bo)   u^H - u^H_old of coarse plane zo at
//                           byte offset bo
//   k.add_corr(cell, v)     the cell with the correction v added to its state
// Every global load and store is issued by every lane (masked cells use an
// out-of-range offset), so the loads in flight for later steps are never
// waited for early.
#pragma once

#include <type_traits>

#include "device_common.h"

namespace vmg {

// Threads per block of the fused sweep: one thread per black cell of a tile
// plane (32 TY) for the tall tiles, 256 for the short ones, whose tiles have
// fewer cells than that.
#ifndef VMG_WIDE_TY
#define VMG_WIDE_TY 16
#endif
constexpr int sweep_threads(int ty) { return ty >= VMG_WIDE_TY ? 32 * ty : 256; }

// Pipeline shape (a run-time choice of the schedule, SmoothCfg::pipe).  With
// DEFER the black phase of a step works two planes behind its red phase
// instead of one, so the two phases of a step touch disjoint LDS planes and run
// without a barrier between them (one barrier per step, and red and black
// updates of a thread are independent work); the plane rings then hold four
// planes instead of three.
constexpr int sweep_slots(bool defer) { return defer ? 4 : 3; }

// LDS of a sweep block of tile height TY (8-byte cells: the ring's ring-2
// planes of u^0 and as many ring-1 planes of u^1), and the waves per SIMD its
// kernels are built for: as many blocks per CU as that LDS allows (160 KB per
// CU), at most 4, so that the register budget matches the occupancy the LDS
// permits.
// With the prolongation folded in (pro): four coarse correction planes of the
// tile's window ((TX/2 + 4) x (ty/2 + 4) cells) and two planes of their
// interpolation onto the tile's ring-2 rows ((ty + 4) x (TX/2 + 4)), counted at
// 8 bytes.
constexpr int PRO_SLOTS = 4;
constexpr int pro_window(int ty) { return (TX / 2 + 4) * (ty / 2 + 4); }
constexpr int pro_rows(int ty) { return (TX / 2 + 4) * (ty + 4); }
constexpr int sweep_lds_bytes(int ty, bool defer, bool pro = false) {
    return sweep_slots(defer) * ((TX + 4) * (ty + 4) + (TX + 2) * (ty + 2)) * 8 +
           (pro ? (PRO_SLOTS * pro_window(ty) + 2 * pro_rows(ty)) * 8 : 0);
}
// (at most 4 blocks; with the folded prolongation, whose extra state would not
// fit that register budget, at most 3 for tile height 4 and 2 above)
constexpr int sweep_max_blocks(int ty, bool pro) { return pro ? (ty <= 4 ? 3 : 2) : 4; }
constexpr int sweep_blocks_per_cu(int ty, bool defer, bool pro = false) {
    return (160 * 1024) / sweep_lds_bytes(ty, defer, pro) >= sweep_max_blocks(ty, pro)
               ? sweep_max_blocks(ty, pro)
               : ((160 * 1024) / sweep_lds_bytes(ty, defer, pro) < 1 ? 1
                                                                     : (160 * 1024) / sweep_lds_bytes(ty, defer, pro));
}
// waves per SIMD (the launch bound): the resident blocks' waves over the CU's 4 SIMDs
constexpr int sweep_waves(int ty, bool defer, bool pro = false) {
    return (sweep_blocks_per_cu(ty, defer, pro) * (sweep_threads(ty) / 64) + 3) / 4;
}

// Neighbourhood of a cell read from a parity-split LDS plane set.  `c` is the
// word offset of the cell's row-half position for the neighbours in its own
// x parity class (x-1 at c, x+1 at c+1), `o` the offset of the cell itself in
// the other class (used for the y and z neighbours); W is the row length in
// cells; Pm/Pc/Pp the planes below, at and above the cell.
template <int W, typename T>
__device__ __forceinline__ void nb_split(const T* __restrict__ Pm, const T* __restrict__ Pc,
                                         const T* __restrict__ Pp, int c, int o, NbT<T>& v) {
    v.xm = Pc[c];           v.xp = Pc[c + 1];
    v.xmym = Pc[c - W];     v.xpym = Pc[c - W + 1];
    v.xmyp = Pc[c + W];     v.xpyp = Pc[c + W + 1];
    v.xmzm = Pm[c];         v.xpzm = Pm[c + 1];
    v.xmzp = Pp[c];         v.xpzp = Pp[c + 1];
    v.ym = Pc[o - W];       v.yp = Pc[o + W];
    v.zm = Pm[o];           v.zp = Pp[o];
    v.ymzm = Pm[o - W];     v.ypzm = Pm[o + W];
    v.ymzp = Pp[o - W];     v.ypzp = Pp[o + W];
}

template <int TY, int DIR, int NTH, bool DEFER, bool PRO = false, typename K>
__device__ __forceinline__ void fused_sweep(const K& k, const Geom& g, const int x0, const int y0, const int z0,
                                            const int z1) {
    static_assert(!(PRO && DIR), "the folded prolongation is for periodic grids");
    using Cell = typename K::Cell;
    using Src = typename K::Src;
    static_assert(sizeof(Cell) == 8, "sweep_lds_bytes assumes 8-byte cells");
    constexpr int W2 = TX + 4, H2 = TY + 4, W1 = TX + 2, H1 = TY + 2;
    constexpr int HW2 = W2 / 2, HW1 = W1 / 2;     // half-row lengths (34, 33)
    constexpr int NP2 = W2 * H2;
    constexpr int NL2 = (NP2 + NTH - 1) / NTH;
    constexpr int RH = W1 / 2;        // red/black pairs per ring-1 row (33)
    static_assert(RH == 33, "the red slot mapping assumes 33 pairs per ring-1 row");
    constexpr int BH = TX / 2;        // black cells per interior row
    constexpr int NR = (RH * H1 + NTH - 1) / NTH;   // red cells per thread
    constexpr int NB = (BH * TY + NTH - 1) / NTH;   // black cells per thread
    constexpr int S2 = H2 * W2, S1 = H1 * W1;     // cells per plane
    // Rows are stored split by x parity: cell (Y, X) lives at Y*W + (X&1)*W/2 + (X>>1),
    // so lanes working on every other cell of a row touch consecutive words.
    constexpr int NSL = sweep_slots(DEFER), LAG = DEFER ? 3 : 2;
    __shared__ Cell P0[NSL * S2];  // u^0, ring 2, slot = z mod NSL
    __shared__ Cell P1[NSL * S1];  // u^1 (red computed, black copied), ring 1

    const int tid = threadIdx.x;
    if (z0 >= g.n2) return;
    constexpr int EB = K::EB;
    // in-plane offsets are taken from the grid's own storage start (a pooled
    // batch adds g.base to the plane resources instead)
    const int64_t loff0 = g.off0 - g.base;

    // ---- per-thread constants (everything that does not depend on z) -------
    int ob2[NL2], lds2[NL2];   // byte offset in a plane of u^0 (out of range: zero), LDS word
#pragma unroll
    for (int s = 0; s < NL2; ++s) {
        const int e = tid + s * NTH;
        ob2[s] = BUF_OOB;
        lds2[s] = 0;
        if (e < NP2) {
            const int X = e % W2, Y = e / W2;
            lds2[s] = Y * W2 + (X & 1) * HW2 + (X >> 1);
            int gx = x0 - 2 + X, gy = y0 - 2 + Y;
            bool ok = true;
            if (DIR) {
                ok = gx >= -1 && gx <= g.n0 && gy >= -1 && gy <= g.n1;
            } else {
                gx = wrapi(gx, g.n0);
                gy = wrapi(gy, g.n1);
            }
            if (ok) ob2[s] = (int)(loff0 + gx + (int64_t)gy * g.sy) * EB;
        }
    }
    // ---- folded prolongation (PRO) --------------------------------------------
    // u^0 = u^h + P(u^H - u^H_old) is formed as the planes are staged: each
    // ring-2 cell adds the cell-centred trilinear interpolation (weights 3/4 and
    // 1/4 per axis) of the coarse correction.  The tile's ring-2 cells draw on the
    // coarse window cx0 .. cx0 + CW - 1, cy0 .. cy0 + CH - 1 (cx0 = x0/2 - 2,
    // cy0 = y0/2 - 2; x0, y0 even); coarse plane K of the window sits in slot
    // K & 3 of PC.  A fine plane p needs coarse planes p >> 1 and (p >> 1) -+ 1
    // (p even / odd).  The interpolation is separable: for plane p, EY (slot
    // p & 1) first holds the z- and y-interpolated window column of every ring-2
    // row; a cell then needs two of them.
    using Corr = typename K::Corr;
    constexpr int CW = TX / 2 + 4, CH = TY / 2 + 4, CWH = CW * CH, EYS = H2 * CW;
    constexpr int NCW = PRO ? (CWH + NTH - 1) / NTH : 1;
    constexpr int NEY = PRO ? (EYS + NTH - 1) / NTH : 1;
    constexpr int NPB = PRO ? NL2 : 1;
    __shared__ Corr PC[PRO ? PRO_SLOTS * CWH : 1];
    __shared__ Corr EY[PRO ? 2 * EYS : 1];
    int cob[NCW], cl[NCW];   // byte offset of a window cell in a coarse plane, its LDS word (-1: none)
    int eyo[NEY], eyd[NEY];  // EY entry: window word of (J, column) (-1: none), y step (+-CW)
    int pwin[NPB][2];        // ring-2 cell: EY word of (row, I), x step (+-1)
    if (PRO) {
#pragma unroll
        for (int q = 0; q < NCW; ++q) {
            const int e = tid + q * NTH;
            cl[q] = e < CWH ? e : -1;
            cob[q] = BUF_OOB;
            if (e < CWH) {
                const int I = wrapi((x0 >> 1) - 2 + e % CW, k.gc.n0), J = wrapi((y0 >> 1) - 2 + e / CW, k.gc.n1);
                cob[q] = (int)(k.gc.off0 - k.gc.base + I + (int64_t)J * k.gc.sy) * EB;
            }
        }
#pragma unroll
        for (int q = 0; q < NEY; ++q) {
            const int e = tid + q * NTH;
            const int Y = e / CW, c = e % CW;      // ring-2 row, window column
            eyo[q] = e < EYS ? (1 + (Y >> 1)) * CW + c : -1;
            eyd[q] = (Y & 1) ? CW : -CW;
        }
#pragma unroll
        for (int s = 0; s < NPB; ++s) {
            const int e = tid + s * NTH;
            const int X = e < NP2 ? e % W2 : 0, Y = e < NP2 ? e / W2 : 0;
            pwin[s][0] = Y * CW + 1 + (X >> 1);
            pwin[s][1] = (X & 1) ? 1 : -1;
        }
    }
    auto coarse_load = [&](int kc, Corr (&v)[NCW]) {
        const auto C = k.coarse_plane(k.gc.base + (int64_t)wrapi(kc, k.gc.n2) * k.gc.sz);
#pragma unroll
        for (int q = 0; q < NCW; ++q) v[q] = k.coarse_b(C, cob[q]);
    };
    auto coarse_store = [&](int kc, const Corr (&v)[NCW]) {
        Corr* dst = PC + (kc & (PRO_SLOTS - 1)) * CWH;
#pragma unroll
        for (int q = 0; q < NCW; ++q)
            if (cl[q] >= 0) dst[cl[q]] = v[q];
    };
    // EY of fine plane p from its two coarse planes (z, then y)
    auto make_ey = [&](int p) {
        const int kp = p >> 1, sk = (p & 1) ? 1 : -1;
        const Corr* C0 = PC + (kp & (PRO_SLOTS - 1)) * CWH;
        const Corr* C1 = PC + ((kp + sk) & (PRO_SLOTS - 1)) * CWH;
        Corr* E = EY + (p & 1) * EYS;
        const Corr a = Corr(0.75), b = Corr(0.25);
#pragma unroll
        for (int q = 0; q < NEY; ++q) {
            if (eyo[q] < 0) continue;
            const int o = eyo[q], dy = eyd[q];
            const Corr z0v = a * C0[o] + b * C1[o];
            const Corr z1v = a * C0[o + dy] + b * C1[o + dy];
            E[tid + q * NTH] = a * z0v + b * z1v;
        }
    };
    // the correction of plane p (its EY written and synchronised) at this
    // thread's ring-2 cells, and its addition to the staged cells
    auto read_prolonged = [&](int p, Corr (&v)[NPB]) {
        const Corr* E = EY + (p & 1) * EYS;
        const Corr a = Corr(0.75), b = Corr(0.25);
#pragma unroll
        for (int s = 0; s < NPB; ++s) {
            const int o = pwin[s][0];
            v[s] = a * E[o] + b * E[o + pwin[s][1]];
        }
    };
    auto add_prolonged = [&](const Corr (&v)[NPB], Cell (&r)[NL2]) {
#pragma unroll
        for (int s = 0; s < NPB; ++s)
            if (tid + s * NTH < NP2) r[s] = k.add_corr(r[s], v[s]);
    };

    // The loop below is unrolled twice, so step t = z0 + 2k + b works on planes
    // of fixed parity per b: red on p = t - 1, black on p2 = t - 2.  Every
    // parity-dependent offset is therefore chosen once here, per b.
    const int zpar = z0 & 1;
    // The two parities of a slot's column are swapped between b = 0 and b = 1,
    // so several per-b offsets coincide with the other b's partner offsets
    // (the cell itself at parity par is the partner's source at 1 - par); only
    // one copy of each is kept.
    // red cells: ring-1 row r, pair m; parity par = (y0 + r + p) & 1 puts the red cell at
    // ring-1 column 2m + par and the black one at 2m + 1 - par
    bool rv[NR];              // slot exists
    int rc[NR][2], ro[NR][2]; // nb_split offsets in P0 (ring 2), per b; ro[q][1-b] is also
                              // the P0 cell of step b's black partner (copied into P1)
    int rw[NR][2];            // P1 cell of step b's red cell; rw[q][1-b] holds its black partner
    int rg[NR][2];            // global in-plane index of the red cell (-1: not a cell)
    int rgb[NR][2];           // its byte offset in a source plane (out of range: not a cell)
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        const int e = tid + q * NTH;
        rv[q] = e < RH * H1;
        // pairs 0..31 of every row take 32 consecutive threads, so a 16-lane LDS
        // access group never straddles two rows (no bank conflicts); the last
        // pair of each row (m = 32) goes to the threads after them
        const bool main_part = e < 32 * H1;
        const int r = !rv[q] ? 0 : (main_part ? e >> 5 : e - 32 * H1);
        const int m = !rv[q] ? 0 : (main_part ? (e & 31) : 32);
        const int gy = y0 - 1 + r;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int par = (y0 + r + zpar + b + 1) & 1;
            const int Y = r + 1;                                  // ring-2 row
            rc[q][b] = Y * W2 + par * HW2 + m;                    // x-1 of the red cell (X = 2m+par+1)
            ro[q][b] = Y * W2 + (1 - par) * HW2 + m + par;        // the red cell itself
            rw[q][b] = r * W1 + par * HW1 + m;                    // ring-1 column 2m+par
            int gx = x0 - 1 + 2 * m + par, wy = gy;
            if (DIR) {
                rg[q][b] = (rv[q] && gx >= 0 && gx < g.n0 && gy >= 0 && gy < g.n1)
                               ? (int)(loff0 + gx + (int64_t)gy * g.sy) : -1;
            } else {
                gx = wrapi(gx, g.n0);
                wy = wrapi(gy, g.n1);
                rg[q][b] = rv[q] ? (int)(gx + (int64_t)wy * g.sy) : -1;
            }
            rgb[q][b] = rg[q][b] >= 0 ? rg[q][b] * EB : BUF_OOB;
        }
    }
    // black cells: interior row r, pair m; black at column 2m + ((y0 + r + p2 + 1) & 1).
    // With more threads than black cells, the black cells go to the highest
    // waves so that red and black work land on different waves.
    constexpr int BOFF = NTH > BH * TY ? ((NTH - BH * TY) / 64) * 64 : 0;
    const int tb = tid - BOFF;
    int bc[NB][2], bo[NB][2];   // nb_split offsets in P1, per b; bo[q][1-b] is the red partner
    int bcb[NB][2];             // byte offset of the black cell in a plane ([1-b]: its red
                                // partner); out of range when that cell is not in the grid
    bool bin[NB][2];            // that cell lies inside the grid
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int e = tb + q * NTH;
        const bool slot = e >= 0 && e < BH * TY;                  // a black cell of the tile
        const int r = slot ? e / BH : 0, m = slot ? e - r * BH : 0;   // (0, 0) keeps LDS reads in range
        const int gy = y0 + r;
        const bool bv = slot && gy < g.n1;
        const int row = (int)(loff0 + (int64_t)gy * g.sy) + x0 + 2 * m;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int par = (y0 + r + zpar + b + 1) & 1;
            const int Y = r + 1;                                   // ring-1 row
            bc[q][b] = Y * W1 + par * HW1 + m;                     // x-1 of the black cell (X = 2m+par+1)
            bo[q][b] = Y * W1 + (1 - par) * HW1 + m + par;         // the black cell itself
            bin[q][b] = bv && 2 * m + par < g.n0 - x0;
            bcb[q][b] = bin[q][b] ? (row + par) * EB : BUF_OOB;
        }
    }
    // element offset of plane t of the grid (storage start included) and whether it
    // exists (Dirichlet: the ghost planes -1 and n2 do; periodic planes wrap)
    auto plane_off = [&](int t, bool& zok) -> int64_t {
        int gz;
        if (DIR) { gz = t; zok = t >= -1 && t <= g.n2; }
        else { gz = t < 0 ? t + g.n2 : (t >= g.n2 ? t - g.n2 : t); zok = true; }
        return g.base + (int64_t)gz * g.sz;
    };
    // `use` false (uniform): the accesses are still issued but read zero, so every
    // step issues the same memory instructions whether or not its planes exist
    auto load_plane = [&](int t, bool use, Cell (&r)[NL2]) {
        bool zok;
        const int64_t zo = plane_off(t, zok);
        const auto P = k.in_plane(use ? zo : g.base, zok && use);
#pragma unroll
        for (int s = 0; s < NL2; ++s) r[s] = k.cell_b(P, ob2[s]);
    };
    auto store_plane = [&](int sl, const Cell (&r)[NL2]) {
#pragma unroll
        for (int s = 0; s < NL2; ++s)
            if (tid + s * NTH < NP2) P0[sl * S2 + lds2[s]] = r[s];
    };
    auto slot = [](int z) { return (z + 3 * NSL) % NSL; };   // z >= -3 NSL

    // sources of the red cells of plane p, whose parity is that of step b's red plane
    auto fetch_red = [&](int p, bool use, auto btag, Src (&sr)[NR]) {
        constexpr int b = decltype(btag)::value;
        bool zok;
        const int64_t zo = plane_off(p, zok);
        if (DIR) zok = p >= 0 && p < g.n2;
        const auto S = k.src_plane(use ? zo : g.base, zok && use);
#pragma unroll
        for (int q = 0; q < NR; ++q) sr[q] = k.src_b(S, rgb[q][b]);
    };
    // sources of the black cells of plane p2, whose parity is that of step b's black plane
    auto fetch_black = [&](int p2, bool use, auto btag, Src (&sr)[NB]) {
        constexpr int b = decltype(btag)::value;
        const auto S = k.src_plane(use ? g.base + (int64_t)p2 * g.sz : g.base, use);
#pragma unroll
        for (int q = 0; q < NB; ++q) sr[q] = k.src_b(S, bcb[q][b]);
    };
    using B0 = std::integral_constant<int, 0>;
    using B1 = std::integral_constant<int, 1>;

    // ---- red phase on plane p, ring 1: P0 -> P1 (sources sr of plane p) -----
    auto red_phase = [&](const int p, auto btag, const Src (&sr)[NR]) {
        constexpr int b = decltype(btag)::value;
        const Cell* Pm = P0 + slot(p - 1) * S2;
        const Cell* Pc = P0 + slot(p) * S2;
        const Cell* Pp = P0 + slot(p + 1) * S2;
        Cell* Q1 = P1 + slot(p) * S1;
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            if (!rv[q]) continue;
            const int c = rc[q][b], o = ro[q][b];
            Cell val = Pc[o];
            const bool interior = DIR ? (rg[q][b] >= 0 && p >= 0 && p < g.n2) : true;
            if (interior) val = k.template update<W2>(Pm, Pc, Pp, c, o, sr[q]);
            Q1[rw[q][b]] = val;
            Q1[rw[q][1 - b]] = Pc[ro[q][1 - b]];
        }
    };
    // ---- black phase on plane p2, tile interior: P1 -> u^2 (sources sr) ------
    auto black_phase = [&](const int p2, auto btag, const Src (&sr)[NB]) {
        constexpr int b = decltype(btag)::value;
        const Cell* Rm = P1 + slot(p2 - 1) * S1;
        const Cell* Rc = P1 + slot(p2) * S1;
        const Cell* Rp = P1 + slot(p2 + 1) * S1;
        const auto O = k.out_plane(g.base + (int64_t)p2 * g.sz, true);
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            Cell v = Rc[bo[q][b]];
            if (bin[q][b]) v = k.template update<W1>(Rm, Rc, Rp, bc[q][b], bo[q][b], sr[q]);
            k.out_b(O, bcb[q][b], v);
            k.out_b(O, bcb[q][1 - b], Rc[bo[q][1 - b]]);
        }
    };

    // Software pipeline over z.  Step t computes red on plane t-1 (u^0 planes
    // t-2..t in LDS) and black on plane t-LAG (u^1 planes t-LAG-1..t-LAG+1 in
    // LDS).  LAG = 2: the black phase reads the red phase's plane, so a barrier
    // separates them; LAG = 3: the phases touch disjoint planes of the four-plane
    // rings and a step has one barrier.  The loop body is unrolled twice, so
    // parity-dependent offsets and buffer indices are compile-time selections.
    // K::AHEAD sets how far loads run ahead of their use:
    //   2: the u^0 plane t+2 is issued at the start of step t and committed to
    //      LDS at the end of step t+1; sources are issued two steps before use
    //      (register buffers alternate with the step's parity);
    //   1: the u^0 plane t+1 is issued at the start of step t and committed at
    //      its end; the next step's sources are issued right after the phase
    //      that consumed the buffer (half the registers).
    // The steps without a black plane (the first LAG) and, with LAG = 3, the last
    // step (no red plane) are peeled off, so the loop body issues the same loads
    // and stores every step (loads of planes past the chunk read zero through an
    // empty resource).
    static_assert(K::AHEAD == 1 || K::AHEAD == 2, "pipeline depth 1 or 2");
    constexpr int NBUF = K::AHEAD;
    Cell pq[NBUF][NL2];     // u^0 planes in flight
    Src rq[NBUF][NR];       // red sources
    Src bq[NBUF][NB];       // black sources
    Corr cq[NCW];           // PRO: coarse plane in flight (issued on even steps)
    if (PRO) {
        // coarse planes z0/2 - 2 .. z0/2 + 1: those of fine planes z0 - 2 .. z0 + 2
        Corr cv[PRO_SLOTS][NCW];
#pragma unroll
        for (int j = 0; j < PRO_SLOTS; ++j) coarse_load((z0 >> 1) - 2 + j, cv[j]);
#pragma unroll
        for (int j = 0; j < PRO_SLOTS; ++j) coarse_store((z0 >> 1) - 2 + j, cv[j]);
        __syncthreads();
    }
    {
        Cell r2[NL2];
        for (int t = z0 - 2; t <= z0; ++t) {
            load_plane(t, true, r2);
            if (PRO) {
                make_ey(t);
                __syncthreads();
                Corr v[NPB];
                read_prolonged(t, v);
                add_prolonged(v, r2);
            }
            store_plane(slot(t), r2);
        }
        if (PRO) make_ey(z0 + 1);   // stored by step z0
        if (K::AHEAD == 2) {
            load_plane(z0 + 1, true, pq[NBUF - 1]);
            fetch_red(z0, true, B1(), rq[NBUF - 1]);   // red plane of step z0 + 1
        }
        fetch_red(z0 - 1, true, B0(), rq[0]);          // red plane of step z0
    }
    __syncthreads();

    // parity class (for the black offsets) of black plane pl: (pl - z0) & 1
    auto step = [&](const int t, auto parity_tag, auto red_tag, auto black_tag) {
        constexpr int b = decltype(parity_tag)::value;
        constexpr bool RED = decltype(red_tag)::value;      // a red plane (t - 1 <= z1)
        constexpr bool BLACK = decltype(black_tag)::value;  // a black plane (t - LAG >= z0)
        using BN = std::integral_constant<int, 1 - b>;       // parity of step t+1
        // black offsets of plane t - LAG: class b for LAG = 2, 1 - b for LAG = 3
        using BB = std::integral_constant<int, LAG == 2 ? b : 1 - b>;
        constexpr int cur = K::AHEAD == 2 ? b : 0;            // buffers used by this step
        const int p = t - 1, pb = t - LAG;
        // PRO: step t forms EY of fine plane t + 2 (stored by step t + 1) in slot
        // t & 1, whose last reader was step t - 1.  An even step (z0 is even)
        // issues coarse plane t/2 + 2, first read by step t + 1; its slot last
        // served EY of plane t - 2.
        constexpr bool CLOAD = PRO && b == 0;
        if (RED && CLOAD) coarse_load((t >> 1) + 2, cq);
        if (RED && PRO) make_ey(t + 2);
        // correction of plane t + 1, read early so that its LDS latency is hidden
        Corr pv[NPB];
        if (RED && PRO) read_prolonged(t + 1, pv);
        if (RED) {
            if (K::AHEAD == 2)
                load_plane(t + 2, t + 2 <= z1 + 1, pq[cur]);
            else
                load_plane(t + 1, t + 1 <= z1 + 1, pq[0]);
            red_phase(p, parity_tag, rq[cur]);
            if (K::AHEAD == 2)
                fetch_red(t + 1, t + 1 <= z1, parity_tag, rq[cur]);   // plane t+1 has the parity of t-1
            else
                fetch_red(t, t <= z1, BN(), rq[0]);                   // red plane of step t+1
        }
        if (LAG == 2) __syncthreads();
        if (BLACK) black_phase(pb, BB(), bq[cur]);
        if (RED) {
            // sources of the black plane of step t + AHEAD (plane t + AHEAD - LAG)
            const int pn = t + K::AHEAD - LAG;
            using BNX = std::integral_constant<int, ((K::AHEAD - LAG) & 1) ? 1 - b : b>;
            fetch_black(pn, pn >= z0 && pn < z1, BNX(), bq[cur]);
            // commit u^0 plane t+1 (its slot is read by no phase of this step; past
            // the chunk's last red step the slot is never read again)
            if (PRO) add_prolonged(pv, pq[K::AHEAD == 2 ? (b ^ 1) : 0]);
            store_plane(slot(t + 1), pq[K::AHEAD == 2 ? (b ^ 1) : 0]);
            if (CLOAD) coarse_store((t >> 1) + 2, cq);
        }
        __syncthreads();
    };
    using Yes = std::true_type;
    using No = std::false_type;
    step(z0, B0(), Yes(), No());
    step(z0 + 1, B1(), Yes(), No());
    int t = z0 + 2;
    if (LAG == 2) {
        for (; t + 1 <= z1 + 1; t += 2) {
            step(t, B0(), Yes(), Yes());
            step(t + 1, B1(), Yes(), Yes());
        }
        if (t <= z1 + 1) step(t, B0(), Yes(), Yes());
    } else {
        step(t, B0(), Yes(), No());
        for (t = z0 + 3; t + 1 <= z1 + 1; t += 2) {
            step(t, B1(), Yes(), Yes());
            step(t + 1, B0(), Yes(), Yes());
        }
        if (t <= z1 + 1) {
            step(t, B1(), Yes(), Yes());
            ++t;
        }
        // last step: black on plane z1 - 1 only
        if (((t - z0) & 1) == 0)
            step(t, B0(), No(), Yes());
        else
            step(t, B1(), No(), Yes());
    }
}

// ---------------------------------------------------------------------------
// Several sweeps of a small periodic level in one launch, without the z march
// (the march's pipeline fill dominates there).  A block owns a BB^3 brick and
// runs S red-black sweeps (S = 1 or 2) of it: it stages u^0 on a ring of 2S
// cells around the brick (periodic wrap) and the sources on a ring of 2S - 1;
// phase p = 2 s + colour (sweep s, red then black) updates the cells of that
// colour within ring 2S - 1 - p of the brick, so each phase finds its
// neighbourhood complete from the previous phases and no block reads another
// block's output (the rings are recomputed, as in the march).  A phase forms its
// updates in registers and writes them in place after a barrier: the red phase
// reads u^0 only (same-colour edge neighbours included), the black phase the
// state with that sweep's reds updated, so the sweeps are those of the march.
// With PRO the staged state first gets the prolonged coarse correction, with
// the folded march's interpolation order (z, then y, then x).
// DIR = 1: a padded Dirichlet level (one sweep, S = 1): the region is staged
// from the stored cells and ghost shell (what lies beyond the shell is never a
// neighbour of an interior cell and stages as zero), and only interior cells
// are updated: the ghosts are the sweep's boundary values.  With GHOSTS the
// output's ghost shell is refreshed as the brick goes out (coarse levels, whose
// ghosts follow the interior: k.store_ghost).
//
// Policy interface (besides Cell, Src, Corr, add_corr and gc of the march):
//   k.load_cell(i), k.load_src(i), k.store_cell(i, v)   element i of the level
//   k.load_corr(i)                  u^H - u^H_old at element i of the coarse level
//   k.update_nb(v, centre, src)     the updated cell from its 18 neighbours
// ---------------------------------------------------------------------------
constexpr int BB = BB_SIDE;
constexpr int BRICK_THREADS = 512;
constexpr int BRICK_WAVES = 4;   // waves per SIMD: two blocks per CU (LDS <= 80 KB each)
constexpr int brick_side(int s) { return BB + 4 * s; }          // staged region, per axis
constexpr int brick_cwin(int s) { return brick_side(s) / 2 + 2; }   // coarse window, per axis

__device__ __forceinline__ int wrap_idx(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

// whether padded element (x, y, z) of a Dirichlet level is stored (ghost shell included)
__device__ __forceinline__ bool in_shell(const Geom& g, int x, int y, int z) {
    return x >= -1 && x <= g.n0 && y >= -1 && y <= g.n1 && z >= -1 && z <= g.n2;
}

// Refresh the face and edge ghosts of the output whose mirrored interior cell is
// (x, y, z) (element ii), from its new value v: each ghost has one such cell,
// and the sign flips once per mirrored axis.
template <typename K, typename Cell>
__device__ __forceinline__ void brick_store_ghosts(const K& k, const Geom& g, int x, int y, int z, int64_t ii,
                                                   const Cell& v) {
    if (x > 0 && x < g.n0 - 1 && y > 0 && y < g.n1 - 1 && z > 0 && z < g.n2 - 1) return;
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                const int out = (dx != 0) + (dy != 0) + (dz != 0);
                if (out == 0 || out == 3) continue;   // the cell itself; corners are not stored
                const int gx = x + dx, gy = y + dy, gz = z + dz;
                if ((dx != 0 && gx >= 0 && gx < g.n0) || (dy != 0 && gy >= 0 && gy < g.n1) ||
                    (dz != 0 && gz >= 0 && gz < g.n2))
                    continue;                         // a step that stays inside: not a ghost of this cell
                k.store_ghost(cell_index(g, gx, gy, gz), ii, out == 1 ? -1 : 1, v);
            }
}

template <int S, bool PRO, int DIR = 0, bool GHOSTS = false, typename K>
__device__ __forceinline__ void brick_sweeps(const K& k, const Geom& g, int bx0, int by0, int bz0) {
    using Cell = typename K::Cell;
    using Src = typename K::Src;
    using Corr = typename K::Corr;
    constexpr int NTH = BRICK_THREADS;
    constexpr int R = 2 * S;                   // staged ring
    constexpr int RW = brick_side(S), RW2 = RW * RW, NU = RW2 * RW;
    constexpr int RS = RW - 2, NS = RS * RS * RS;   // sources on ring 2S - 1
    constexpr int CW = brick_cwin(S), NCW = CW * CW * CW;
    constexpr int NLU = (NU + NTH - 1) / NTH, NLS = (NS + NTH - 1) / NTH;
    constexpr int NQ = (NS / 2 + NTH - 1) / NTH;   // widest phase: one colour of ring 2S - 1
    static_assert(!PRO || NCW * sizeof(Corr) <= NU * sizeof(Cell), "the coarse window lives in U's space");
    static_assert(!DIR || (S == 1 && !PRO), "Dirichlet levels: one sweep, no folded prolongation");
    static_assert(!GHOSTS || DIR, "only Dirichlet levels have a ghost shell");
    __shared__ Cell U[NU];
    __shared__ Src SR[NS];
    // the coarse window is read before U is written: it borrows U's space
    Corr* CWB = reinterpret_cast<Corr*>(U);
    const int tid = threadIdx.x;

    // ---- staging: u^0 (+ prolonged correction) on ring 2S, sources on ring 2S - 1
    Cell u0[NLU];
#pragma unroll
    for (int q = 0; q < NLU; ++q) {
        const int e = tid + q * NTH;
        if (e < NU) {
            const int x = e % RW, y = (e / RW) % RW, z = e / RW2;
            if (DIR) {
                const int gx = bx0 - R + x, gy = by0 - R + y, gz = bz0 - R + z;
                u0[q] = in_shell(g, gx, gy, gz) ? k.load_cell(cell_index(g, gx, gy, gz)) : Cell{};
            } else {
                u0[q] = k.load_cell(cell_index(g, wrap_idx(bx0 - R + x, g.n0), wrap_idx(by0 - R + y, g.n1),
                                               wrap_idx(bz0 - R + z, g.n2)));
            }
        }
    }
    // every load is issued before the first LDS write (registers, then LDS)
    Src s0[NLS];
#pragma unroll
    for (int q = 0; q < NLS; ++q) {
        const int e = tid + q * NTH;
        if (e < NS) {
            const int x = e % RS, y = (e / RS) % RS, z = e / (RS * RS);
            if (DIR) {
                const int gx = bx0 - R + 1 + x, gy = by0 - R + 1 + y, gz = bz0 - R + 1 + z;
                s0[q] = in_shell(g, gx, gy, gz) ? k.load_src(cell_index(g, gx, gy, gz)) : Src{};
            } else {
                s0[q] = k.load_src(cell_index(g, wrap_idx(bx0 - R + 1 + x, g.n0), wrap_idx(by0 - R + 1 + y, g.n1),
                                              wrap_idx(bz0 - R + 1 + z, g.n2)));
            }
        }
    }
    constexpr int NLC = PRO ? (NCW + NTH - 1) / NTH : 1;
    Corr c0[NLC];
    if (PRO) {
        // coarse window: coarse cells (bx0 - R) / 2 - 1 + [0, CW) per axis (bx0 - R is even)
        const int cx0 = (bx0 - R) / 2 - 1, cy0 = (by0 - R) / 2 - 1, cz0 = (bz0 - R) / 2 - 1;
#pragma unroll
        for (int q = 0; q < NLC; ++q) {
            const int e = tid + q * NTH;
            if (e < NCW) {
                const int x = e % CW, y = (e / CW) % CW, z = e / (CW * CW);
                c0[q] = k.load_corr(cell_index(k.gc, wrap_idx(cx0 + x, k.gc.n0), wrap_idx(cy0 + y, k.gc.n1),
                                               wrap_idx(cz0 + z, k.gc.n2)));
            }
        }
    }
#pragma unroll
    for (int q = 0; q < NLS; ++q) {
        const int e = tid + q * NTH;
        if (e < NS) SR[e] = s0[q];
    }
    if (PRO) {
#pragma unroll
        for (int q = 0; q < NLC; ++q) {
            const int e = tid + q * NTH;
            if (e < NCW) CWB[e] = c0[q];
        }
        __syncthreads();
        const Corr a = Corr(0.75), b = Corr(0.25);
#pragma unroll
        for (int q = 0; q < NLU; ++q) {
            const int e = tid + q * NTH;
            if (e < NU) {
                const int x = e % RW, y = (e / RW) % RW, z = e / RW2;
                // fine cell x of the region lies in coarse window cell x/2 + 1; its
                // farther coarse neighbour is on the side of its parity
                const int ix = (x >> 1) + 1, iy = (y >> 1) + 1, iz = (z >> 1) + 1;
                const int sx = (x & 1) ? 1 : -1, sy = (y & 1) ? CW : -CW, sz = (z & 1) ? CW * CW : -CW * CW;
                const Corr* C0 = CWB + iz * CW * CW;
                const Corr* C1 = C0 + sz;
                const int o0 = iy * CW + ix, o1 = o0 + sx;
                const Corr z00 = a * C0[o0] + b * C1[o0];
                const Corr z01 = a * C0[o0 + sy] + b * C1[o0 + sy];
                const Corr z10 = a * C0[o1] + b * C1[o1];
                const Corr z11 = a * C0[o1 + sy] + b * C1[o1 + sy];
                const Corr e0 = a * z00 + b * z01;
                const Corr e1 = a * z10 + b * z11;
                u0[q] = k.add_corr(u0[q], a * e0 + b * e1);
            }
        }
        __syncthreads();   // every read of the window is done before U overwrites it
    }
#pragma unroll
    for (int q = 0; q < NLU; ++q) {
        const int e = tid + q * NTH;
        if (e < NU) U[e] = u0[q];
    }
    __syncthreads();

    // ---- the 2S colour phases on shrinking rings
    const int par0 = (bx0 + by0 + bz0) & 1;   // colour of region cell (0,0,0) is par0 (R even)
#pragma unroll
    for (int p = 0; p < 2 * S; ++p) {
        const int colour = p & 1, ring = 2 * S - 1 - p;
        const int lo = R - ring, side = BB + 2 * ring, half = side / 2;
        const int count = half * side * side;
        Cell res[NQ];
        int at[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int e = tid + q * NTH;
            at[q] = -1;
            if (e < count) {
                const int hx = e % half, r = e / half;
                const int y = lo + r % side, z = lo + r / side;
                const int x = lo + 2 * hx + ((colour + par0 + y + z + lo) & 1);
                if (DIR) {
                    const int gx = bx0 - R + x, gy = by0 - R + y, gz = bz0 - R + z;
                    if (gx < 0 || gx >= g.n0 || gy < 0 || gy >= g.n1 || gz < 0 || gz >= g.n2) continue;
                }
                const int c = (z * RW + y) * RW + x;
                NbT<Cell> v;
                v.xm = U[c - 1];                 v.xp = U[c + 1];
                v.ym = U[c - RW];                v.yp = U[c + RW];
                v.zm = U[c - RW2];               v.zp = U[c + RW2];
                v.xmym = U[c - RW - 1];          v.xpym = U[c - RW + 1];
                v.xmyp = U[c + RW - 1];          v.xpyp = U[c + RW + 1];
                v.xmzm = U[c - RW2 - 1];         v.xpzm = U[c - RW2 + 1];
                v.xmzp = U[c + RW2 - 1];         v.xpzp = U[c + RW2 + 1];
                v.ymzm = U[c - RW2 - RW];        v.ypzm = U[c - RW2 + RW];
                v.ymzp = U[c + RW2 - RW];        v.ypzp = U[c + RW2 + RW];
                const Src sv = SR[((z - 1) * RS + (y - 1)) * RS + (x - 1)];
                res[q] = k.update_nb(v, U[c], sv);
                at[q] = c;
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if (at[q] >= 0) U[at[q]] = res[q];
        __syncthreads();
    }

    // ---- the brick (its part inside the level) goes out
    for (int e = tid; e < BB * BB * BB; e += NTH) {
        const int x = e % BB, y = (e / BB) % BB, z = e / (BB * BB);
        const int gx = bx0 + x, gy = by0 + y, gz = bz0 + z;
        if (gx < g.n0 && gy < g.n1 && gz < g.n2) {
            const Cell v = U[((z + R) * RW + (y + R)) * RW + (x + R)];
            const int64_t ii = cell_index(g, gx, gy, gz);
            k.store_cell(ii, v);
            if (GHOSTS) brick_store_ghosts(k, g, gx, gy, gz, ii, v);
        }
    }
}

}  // namespace vmg
