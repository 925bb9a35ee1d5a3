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
//   k.cell(i), k.src(i)     the input state / sources at storage index i
//   k.zero_cell(), k.zero_src()
//   k.template update<W>(Pm, Pc, Pp, c, o, src)   updated cell from its neighbourhood
//   k.out(i, cell)          write the output state at storage index i
#pragma once

#include <type_traits>

#include "device_common.h"

namespace vmg {

// Threads per block of the fused sweep.  Wider blocks measured slower: each
// plane step ends in two block-wide barriers.
constexpr int SNT = 256;

// LDS of a sweep block of tile height TY (8-byte cells: three ring-2 planes of
// u^0 and three ring-1 planes of u^1), and the waves per SIMD its kernels are
// built for: as many blocks per CU as that LDS allows (160 KB per CU), at most
// 4, so that the register budget matches the occupancy the LDS permits.
constexpr int sweep_lds_bytes(int ty) { return 3 * ((TX + 4) * (ty + 4) + (TX + 2) * (ty + 2)) * 8; }
constexpr int sweep_waves(int ty) {
    return (160 * 1024) / sweep_lds_bytes(ty) >= 4 ? 4 : ((160 * 1024) / sweep_lds_bytes(ty) < 1 ? 1 : (160 * 1024) / sweep_lds_bytes(ty));
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

template <int TY, int DIR, int NTH, typename K>
__device__ __forceinline__ void fused_sweep(const K& k, const Geom& g, const int x0, const int y0, const int z0,
                                            const int z1) {
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
    __shared__ Cell P0[3 * S2];  // u^0, ring 2, slot = z mod 3
    __shared__ Cell P1[3 * S1];  // u^1 (red computed, black copied), ring 1

    const int tid = threadIdx.x;
    if (z0 >= g.n2) return;

    // ---- per-thread constants (everything that does not depend on z) -------
    int off2[NL2], lds2[NL2];
    bool ok2[NL2];
#pragma unroll
    for (int s = 0; s < NL2; ++s) {
        const int e = tid + s * NTH;
        ok2[s] = false;
        off2[s] = 0;
        lds2[s] = 0;
        if (e < NP2) {
            const int X = e % W2, Y = e / W2;
            lds2[s] = Y * W2 + (X & 1) * HW2 + (X >> 1);
            int gx = x0 - 2 + X, gy = y0 - 2 + Y;
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
                               ? (int)(g.off0 + gx + (int64_t)gy * g.sy) : -1;
            } else {
                gx = wrapi(gx, g.n0);
                wy = wrapi(gy, g.n1);
                rg[q][b] = rv[q] ? (int)(gx + (int64_t)wy * g.sy) : -1;
            }
        }
    }
    // black cells: interior row r, pair m; black at column 2m + ((y0 + r + p2 + 1) & 1).
    // With more threads than black cells, the black cells go to the highest
    // waves so that red and black work land on different waves.
    constexpr int BOFF = NTH > BH * TY ? ((NTH - BH * TY) / 64) * 64 : 0;
    const int tb = tid - BOFF;
    int bc[NB][2], bo[NB][2];   // nb_split offsets in P1, per b; bo[q][1-b] is the red partner
    int bcell[NB][2];           // in-plane global index of the black cell; [1-b]: its red partner
    bool bin[NB][2];            // that cell lies inside the grid
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int e = tb + q * NTH;
        const int r = e >= 0 ? e / BH : 0, m = e >= 0 ? e - r * BH : 0;
        const int gy = y0 + r;
        const bool bv = e >= 0 && e < BH * TY && gy < g.n1;
        const int row = (int)(g.off0 + (int64_t)gy * g.sy) + x0 + 2 * m;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int par = (y0 + r + zpar + b + 1) & 1;
            const int Y = r + 1;                                   // ring-1 row
            bc[q][b] = Y * W1 + par * HW1 + m;                     // x-1 of the black cell (X = 2m+par+1)
            bo[q][b] = Y * W1 + (1 - par) * HW1 + m + par;         // the black cell itself
            bcell[q][b] = row + par;
            bin[q][b] = bv && 2 * m + par < g.n0 - x0;
        }
    }
    auto plane_off = [&](int t, bool& zok) -> int64_t {
        int gz;
        if (DIR) { gz = t; zok = t >= -1 && t <= g.n2; }
        else { gz = t < 0 ? t + g.n2 : (t >= g.n2 ? t - g.n2 : t); zok = true; }
        return (int64_t)gz * g.sz;
    };
    auto load_plane = [&](int t, Cell (&r)[NL2]) {
        bool zok;
        const int64_t zo = plane_off(t, zok);
#pragma unroll
        for (int s = 0; s < NL2; ++s) r[s] = (ok2[s] && zok) ? k.cell(zo + off2[s]) : k.zero_cell();
    };
    auto store_plane = [&](int sl, const Cell (&r)[NL2]) {
#pragma unroll
        for (int s = 0; s < NL2; ++s)
            if (tid + s * NTH < NP2) P0[sl * S2 + lds2[s]] = r[s];
    };
    auto slot = [](int z) { return (z + 3) % 3; };   // z >= -2

    // sources of the red cells of plane p, whose parity is that of step b's red plane
    auto fetch_red = [&](int p, auto btag, Src (&sr)[NR]) {
        constexpr int b = decltype(btag)::value;
        bool zok;
        int64_t zo = plane_off(p, zok);
        if (DIR) zok = p >= 0 && p < g.n2;
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            const int gi = rg[q][b];
            sr[q] = (zok && gi >= 0) ? k.src(zo + gi) : k.zero_src();
        }
    };
    // sources of the black cells of plane p2, whose parity is that of step b's black plane
    auto fetch_black = [&](int p2, auto btag, Src (&sr)[NB]) {
        constexpr int b = decltype(btag)::value;
        const int64_t zo = (int64_t)p2 * g.sz;
#pragma unroll
        for (int q = 0; q < NB; ++q) sr[q] = bin[q][b] ? k.src(zo + bcell[q][b]) : k.zero_src();
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
        const int64_t zo = (int64_t)p2 * g.sz;
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            if (bin[q][b])
                k.out(zo + bcell[q][b], k.template update<W1>(Rm, Rc, Rp, bc[q][b], bo[q][b], sr[q]));
            if (bin[q][1 - b]) k.out(zo + bcell[q][1 - b], Rc[bo[q][1 - b]]);
        }
    };

    // Software pipeline over z.  Step t computes red on plane t-1 (u^0 planes
    // t-2..t in LDS) and black on plane t-2 (u^1 planes t-3..t-1 in LDS).  The
    // loop body is unrolled twice, so parity-dependent offsets and buffer
    // indices are compile-time selections.  K::AHEAD sets how far loads run
    // ahead of their use:
    //   2: the u^0 plane t+2 is issued at the start of step t and committed to
    //      LDS at the end of step t+1; sources are issued two steps before use
    //      (register buffers alternate with the step's parity);
    //   1: the u^0 plane t+1 is issued at the start of step t and committed at
    //      its end; the next plane's sources are issued right after the phase
    //      that consumed the buffer (half the registers).
    static_assert(K::AHEAD == 1 || K::AHEAD == 2, "pipeline depth 1 or 2");
    constexpr int NBUF = K::AHEAD;
    Cell pq[NBUF][NL2];     // u^0 planes in flight
    Src rq[NBUF][NR];       // red sources
    Src bq[NBUF][NB];       // black sources
    {
        Cell r2[NL2];
        for (int t = z0 - 2; t <= z0; ++t) {
            load_plane(t, r2);
            store_plane(slot(t), r2);
        }
        if (K::AHEAD == 2) {
            load_plane(z0 + 1, pq[NBUF - 1]);
            fetch_red(z0, B1(), rq[NBUF - 1]);   // red plane of step z0 + 1
        }
        fetch_red(z0 - 1, B0(), rq[0]);          // red plane of step z0
    }
    __syncthreads();

    auto step = [&](const int t, auto parity_tag) {
        constexpr int b = decltype(parity_tag)::value;
        using BN = std::integral_constant<int, 1 - b>;   // parity of step t+1
        constexpr int cur = K::AHEAD == 2 ? b : 0;        // buffers used by this step
        const int p = t - 1, p2 = t - 2;
        if (K::AHEAD == 2) {
            if (t + 2 <= z1 + 1) load_plane(t + 2, pq[cur]);
        } else {
            if (t + 1 <= z1 + 1) load_plane(t + 1, pq[0]);
        }
        red_phase(p, parity_tag, rq[cur]);
        if (K::AHEAD == 2) {
            if (t + 1 <= z1) fetch_red(t + 1, parity_tag, rq[cur]);   // plane t+1 has the parity of t-1
        } else {
            if (t <= z1) fetch_red(t, BN(), rq[0]);                  // red plane of step t+1
        }
        __syncthreads();
        if (p2 >= z0) black_phase(p2, parity_tag, bq[cur]);
        if (K::AHEAD == 2) {
            if (t >= z0 && t < z1) fetch_black(t, parity_tag, bq[cur]);   // plane t has the parity of t-2
        } else {
            if (t - 1 >= z0 && t - 1 < z1) fetch_black(t - 1, BN(), bq[0]);   // black plane of step t+1
        }
        // ---- commit u^0 plane t+1 (its slot held plane t-2, last read by this red phase)
        if (t + 1 <= z1 + 1) store_plane(slot(t + 1), pq[K::AHEAD == 2 ? (b ^ 1) : 0]);
        __syncthreads();
    };
    int t = z0;
    for (; t + 1 <= z1 + 1; t += 2) {
        step(t, B0());
        step(t + 1, B1());
    }
    if (t <= z1 + 1) step(t, B0());
}

}  // namespace vmg
