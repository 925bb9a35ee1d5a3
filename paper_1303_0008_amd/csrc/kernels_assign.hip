// Mass assignment: unit-mass particles to the density contrast on the periodic
// domain mesh or on a refinement region (Sec. VI: the mesh density comes from
// triangular-shaped-cloud assignment of the particles; cloud in cell is the
// next-lower-order member of the same family of shape functions).  A region is
// not periodic: each particle is taken from the periodic image that reaches
// it, and contributions outside it are dropped.
//
// Both schemes touch the particle's nearest cell and its 26 neighbours at most,
// so the grid is cut into bricks of BRICK^3 cells and every particle belongs to
// the brick of its nearest cell:
//   1. k_bin<0>       particles per brick: each workgroup takes a chunk of
//                     particles, counts them per brick in an LDS hash table and
//                     adds each nonzero count to one of the brick's global
//                     counters (SUB per brick);
//   2. k_scan_*       exclusive prefix sum of the counters;
//   3. k_bin<1>       the same chunks again: each nonzero (chunk, brick) count
//                     reserves a range of that brick's slots with one atomic,
//                     and the particle indices are written sorted by brick;
//   4. k_bin_assign   one workgroup per brick (heaviest bricks first for the
//                     triangular-shaped cloud): the brick and a one-cell halo
//                     are accumulated in LDS and the region is copied to the
//                     workspace;
//   5. k_gather       every cell sums the staged entries of the bricks that
//                     reach it (one; up to 8 on the outer layer of a brick, 27
//                     where bricks are one cell wide) and writes delta.
// No global atomics touch the density, so the sums are formed in a fixed order.
// Masses are 64-bit fixed point (2^-40 of a particle per unit): every
// contribution is rounded once and all sums are integer, so the result does
// not depend on the order of particles or of atomics.
#include <mutex>

#include "device_common.h"
#include "vmg_internal.h"

namespace vmg {
namespace {

constexpr double FIX_ONE = 1099511627776.0;           // 2^40
constexpr double FIX_INV = 1.0 / 1099511627776.0;     // 2^-40
constexpr int BRICK = 16;                             // cells per brick edge
constexpr int REG = BRICK + 2;                        // brick + halo, LDS region edge
constexpr int REGN = REG * REG * REG;
constexpr uint32_t NO_KEY = 0xffffffffu;

struct AGrid {
    int n0, n1, n2;          // cells
    int b0, b1, b2;          // bricks per axis
    // refinement region (not periodic): cell size, corner of cell (0,0,0) and
    // n h + 2h per axis (offsets beyond it belong to the image below the corner)
    double h, cr[3], far[3];
};

// Periodic box: u = position in cells along an axis, in [0, n]; f = floor(u)
// unwrapped; the nearest cell is f mod n.
__device__ __forceinline__ double cells_of(double x, int n) { return (x - floor(x)) * (double)n; }

// Region: the offset from the corner taken modulo 1, moved below the corner
// when it lies beyond the region's far side plus two cells; in cells.
__device__ __forceinline__ double region_u(double x, double corner, double far, double h) {
    double d = x - corner;
    d -= floor(d);
    if (d > far) d -= 1.0;
    return d / h;
}

template <bool PER>
__device__ __forceinline__ double axis_u(const AGrid& g, int a, double x, int n) {
    if constexpr (PER)
        return cells_of(x, n);
    else
        return region_u(x, g.cr[a], g.far[a], g.h);
}

__device__ __forceinline__ bool finite3(double x, double y, double z) {
    return isfinite(x) && isfinite(y) && isfinite(z);
}

// Brick of the particle's nearest cell.  Region: a particle whose nearest cell
// is more than one cell outside reaches no cell of the region (NO_KEY); one
// cell outside, it goes to the brick on that face.
template <bool PER>
__device__ __forceinline__ uint32_t brick_key(const AGrid& g, double x, double y, double z) {
    const double f0 = floor(axis_u<PER>(g, 0, x, g.n0)), f1 = floor(axis_u<PER>(g, 1, y, g.n1)),
                 f2 = floor(axis_u<PER>(g, 2, z, g.n2));
    int c0, c1, c2;
    if constexpr (PER) {
        c0 = (int)f0;
        c1 = (int)f1;
        c2 = (int)f2;
        c0 -= c0 >= g.n0 ? g.n0 : 0;
        c1 -= c1 >= g.n1 ? g.n1 : 0;
        c2 -= c2 >= g.n2 ? g.n2 : 0;
    } else {
        // compared as doubles: far from a small region u can exceed the int range
        if (!(f0 >= -1.0 && f0 <= g.n0 && f1 >= -1.0 && f1 <= g.n1 && f2 >= -1.0 && f2 <= g.n2)) return NO_KEY;
        c0 = min(max((int)f0, 0), g.n0 - 1);
        c1 = min(max((int)f1, 0), g.n1 - 1);
        c2 = min(max((int)f2, 0), g.n2 - 1);
    }
    return ((uint32_t)(c2 / BRICK) * g.b1 + (uint32_t)(c1 / BRICK)) * g.b0 + (uint32_t)(c0 / BRICK);
}

// round(a * b) as an integer, for 0 <= a * b < 2^51: the exact product plus
// 2^52 is rounded once (to nearest, ties to even) to a double whose low 52
// mantissa bits hold that integer.
__device__ __forceinline__ unsigned long long fix_round(double a, double b) {
    const double v = fma(a, b, 4503599627370496.0);
    return (unsigned long long)__double_as_longlong(v) & 0x000fffffffffffffull;
}

__global__ void __launch_bounds__(NT) k_fill_u32(uint32_t* __restrict__ p, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT) p[e] = 0u;
}

constexpr int ANT = 512;                              // threads of the brick accumulation
constexpr int SUB = 16;                               // counters per brick (chunk ch uses ch % SUB)
constexpr int CHUNK_PER_THREAD = 8;
constexpr int CHUNK = CHUNK_PER_THREAD * NT;          // particles per chunk
constexpr int TAB = 2 * CHUNK;                        // LDS hash table entries (load <= 1/2)
static_assert(TAB == 1 << 12, "the hash keeps the top 12 bits of the product");

// MODE 0: add every chunk's per-brick counts to counter[] and store each
// particle's brick key.  MODE 1: reserve each chunk's range of every brick's
// slots from counter[] (the cursors) and write the particle indices there.
// Chunk ch counts into sub-counter ch % SUB of a brick, which spreads the
// global atomics of unordered particles over SUB addresses per brick.
// Bricks are found in the LDS table by linear probing from a multiplicative
// hash of the key.
template <int MODE, bool PER>
__global__ void __launch_bounds__(NT) k_bin(AGrid g, const double* __restrict__ pos, int64_t np,
                                            uint32_t* __restrict__ counter, uint32_t* __restrict__ keys,
                                            uint32_t* __restrict__ idx) {
    __shared__ uint32_t tkey[TAB], tcnt[TAB];
    __shared__ uint16_t used[CHUNK];                      // entries this chunk filled, in fill order
    __shared__ uint32_t n_used;
    for (int e = threadIdx.x; e < TAB; e += NT) {
        tkey[e] = NO_KEY;
        tcnt[e] = 0u;
    }
    if (threadIdx.x == 0) n_used = 0u;
    __syncthreads();
    const int64_t nchunk = (np + CHUNK - 1) / CHUNK;
    for (int64_t ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
        uint32_t key[CHUNK_PER_THREAD];
#pragma unroll
        for (int k = 0; k < CHUNK_PER_THREAD; ++k) {
            const int64_t p = ch * CHUNK + k * NT + threadIdx.x;
            key[k] = NO_KEY;
            if (p >= np) continue;
            if (MODE == 0) {
                const double x = pos[3 * p], y = pos[3 * p + 1], z = pos[3 * p + 2];
                if (finite3(x, y, z)) key[k] = brick_key<PER>(g, x, y, z);
                keys[p] = key[k];
            } else {
                key[k] = keys[p];
            }
        }
        // Lanes of a wavefront hold consecutive particles; a run of adjacent
        // lanes with one key is entered by its first lane, which reserves the
        // run's slots with one LDS atomic.
        const int lane = threadIdx.x & 63;
        const unsigned long long below = (2ull << lane) - 1ull;         // lanes 0..lane
        int hs[CHUNK_PER_THREAD];
        uint32_t loc[CHUNK_PER_THREAD];
#pragma unroll
        for (int k = 0; k < CHUNK_PER_THREAD; ++k) {
            const uint32_t prev = (uint32_t)__shfl_up((int)key[k], 1);
            const bool head = lane == 0 || key[k] != prev;
            const unsigned long long heads = __ballot(head);
            const int first = 63 - __clzll(heads & below);               // head of this lane's run
            const unsigned long long after = heads & ~below;
            const int len = (after ? __ffsll(after) - 1 : 64) - lane;    // run length, read by heads only
            int h = -1;
            uint32_t base = 0;
            if (head && key[k] != NO_KEY) {
                h = (int)((key[k] * 2654435761u) >> 20) & (TAB - 1);
                for (;;) {                                // at most CHUNK distinct keys: always a free entry
                    const uint32_t old = atomicCAS(&tkey[h], NO_KEY, key[k]);
                    if (old == NO_KEY) {
                        used[atomicAdd(&n_used, 1u)] = (uint16_t)h;
                        break;
                    }
                    if (old == key[k]) break;
                    h = (h + 1) & (TAB - 1);
                }
                base = atomicAdd(&tcnt[h], (uint32_t)len);
            }
            hs[k] = __shfl(h, first);
            loc[k] = (uint32_t)__shfl((int)base, first) + (uint32_t)(lane - first);
            if (key[k] == NO_KEY) hs[k] = -1;
        }
        __syncthreads();
        const uint32_t sub = (uint32_t)(ch % SUB);
        const int nu = (int)n_used;
        for (int u = threadIdx.x; u < nu; u += NT) {
            const int e = used[u];
            const uint32_t k = tkey[e];
            if (MODE == 0)
                atomicAdd(counter + (size_t)k * SUB + sub, tcnt[e]);
            else
                tcnt[e] = atomicAdd(counter + (size_t)k * SUB + sub, tcnt[e]);   // this chunk's first slot
        }
        if (MODE == 1) {
            __syncthreads();
#pragma unroll
            for (int k = 0; k < CHUNK_PER_THREAD; ++k)
                if (hs[k] >= 0) idx[tcnt[hs[k]] + loc[k]] = (uint32_t)(ch * CHUNK + k * NT + threadIdx.x);
        }
        __syncthreads();
        // empty the filled entries for the next chunk
        for (int u = threadIdx.x; u < nu; u += NT) {
            const int e = used[u];
            tkey[e] = NO_KEY;
            tcnt[e] = 0u;
        }
        __syncthreads();
        if (threadIdx.x == 0) n_used = 0u;
        __syncthreads();
    }
}

// Exclusive prefix sum of the nc counters into start[0..nc] and cursor[0..nc),
// in three launches: per-block sums of SCAN_TILE counters, an exclusive scan
// of those sums in one block, and block-local scans offset by them.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* part, uint32_t* total) {
    const int t = threadIdx.x;
    part[t] = v;
    __syncthreads();
    for (int off = 1; off < NT; off <<= 1) {                 // inclusive Hillis-Steele scan
        const uint32_t u = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += u;
        __syncthreads();
    }
    const uint32_t incl = part[t];
    *total = part[NT - 1];
    __syncthreads();
    return incl - v;
}

constexpr int SCAN_PER_THREAD = 16;
constexpr int SCAN_TILE = SCAN_PER_THREAD * NT;

__global__ void __launch_bounds__(NT) k_scan_sums(const uint32_t* __restrict__ count, int64_t nc,
                                                  uint32_t* __restrict__ sums) {
    __shared__ uint32_t part[NT];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_PER_THREAD;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_PER_THREAD; ++k) s += base + k < nc ? count[base + k] : 0u;
    uint32_t total;
    block_exclusive_scan(s, part, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// One block: exclusive scan of the m tile sums in place (contiguous runs per thread).
__global__ void __launch_bounds__(NT) k_scan_top(uint32_t* __restrict__ sums, int64_t m) {
    __shared__ uint32_t part[NT];
    const int64_t per = (m + NT - 1) / NT;
    const int64_t lo = threadIdx.x * per, hi = lo + per < m ? lo + per : m;
    uint32_t s = 0;
    for (int64_t b = lo; b < hi; ++b) s += sums[b];
    uint32_t total;
    uint32_t run = block_exclusive_scan(s, part, &total);
    for (int64_t b = lo; b < hi; ++b) {
        const uint32_t v = sums[b];
        sums[b] = run;
        run += v;
    }
}

__global__ void __launch_bounds__(NT) k_scan_tiles(const uint32_t* __restrict__ count, int64_t nc,
                                                   const uint32_t* __restrict__ sums, uint32_t* __restrict__ start,
                                                   uint32_t* __restrict__ cursor) {
    __shared__ uint32_t part[NT];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_PER_THREAD;
    uint32_t v[SCAN_PER_THREAD];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_PER_THREAD; ++k) {
        v[k] = base + k < nc ? count[base + k] : 0u;
        s += v[k];
    }
    uint32_t total;
    uint32_t run = sums[blockIdx.x] + block_exclusive_scan(s, part, &total);
#pragma unroll
    for (int k = 0; k < SCAN_PER_THREAD; ++k) {
        if (base + k < nc) {
            start[base + k] = run;
            cursor[base + k] = run;
        }
        run += v[k];
    }
    if (base + SCAN_PER_THREAD >= nc && base < nc) start[nc] = run;    // the thread holding the last counter
}

// Brick-local LDS index of a cell whose brick-local coordinates are l0, l1, l2
// in [-1, BRICK].
__device__ __forceinline__ int reg_index(int l0, int l1, int l2) { return ((l2 + 1) * REG + (l1 + 1)) * REG + (l0 + 1); }

__device__ __forceinline__ bool in_reg(int l) { return (unsigned)(l + 1) <= (unsigned)(BRICK + 1); }

// Per-axis local cells (brick-local coordinate of the first stencil cell) and
// weights.  CIC: weights 1 - t, t on cells floor(u - 1/2) and the next; TSC:
// nearest cell c, d = u - (c + 1/2), weights (1/2 - d)^2/2, 3/4 - d^2,
// (1/2 + d)^2/2 on cells c - 1, c, c + 1.  `org` is the brick's first cell.
template <int M, bool PER>
__device__ __forceinline__ int axis_local(double u, int n, int org, double (&w)[M]) {
    const double f = floor(u);
    int c = (int)f;
    if constexpr (PER) c -= c >= n ? n : 0;               // nearest cell, in this brick (region: may be -1 or n)
    if constexpr (M == 2) {
        const double g = floor(u - 0.5);                  // f - 1 or f
        const double t = (u - 0.5) - g;
        w[0] = 1.0 - t;
        w[1] = t;
        return c - org + (int)(g - f);
    } else {
        const double d = u - (f + 0.5);
        const double a = 0.5 - d, b = 0.5 + d;
        w[0] = 0.5 * (a * a);
        w[1] = 0.75 - d * d;
        w[2] = 0.5 * (b * b);
        return c - org - 1;
    }
}

// Bricks in order of decreasing particle count (64 buckets of 128 particles;
// one block), so the heaviest bricks start first and do not trail the launch
// (used for the triangular-shaped cloud, whose per-particle work makes the
// imbalance worth the extra launch).
constexpr int ORD_NT = 1024;
__global__ void __launch_bounds__(ORD_NT) k_brick_order(const uint32_t* __restrict__ start, int64_t nb,
                                                        uint32_t* __restrict__ order) {
    __shared__ uint32_t hist[64];
    if (threadIdx.x < 64) hist[threadIdx.x] = 0u;
    __syncthreads();
    for (int64_t b = threadIdx.x; b < nb; b += ORD_NT) {
        const uint32_t cnt = start[(b + 1) * SUB] - start[b * SUB];
        atomicAdd(&hist[63 - min(cnt >> 7, 63u)], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int k = 0; k < 64; ++k) {
            const uint32_t v = hist[k];
            hist[k] = run;
            run += v;
        }
    }
    __syncthreads();
    for (int64_t b = threadIdx.x; b < nb; b += ORD_NT) {
        const uint32_t cnt = start[(b + 1) * SUB] - start[b * SUB];
        order[atomicAdd(&hist[63 - min(cnt >> 7, 63u)], 1u)] = (uint32_t)b;
    }
}

template <int M, bool PER>
__global__ void __launch_bounds__(ANT) k_bin_assign(AGrid g, const double* __restrict__ pos,
                                                   const uint32_t* __restrict__ start,
                                                   const uint32_t* __restrict__ idx,
                                                   const uint32_t* __restrict__ order,
                                                   unsigned long long* __restrict__ stage) {
    __shared__ unsigned long long acc[REGN];
    const int key = order ? (int)order[blockIdx.x] : (int)blockIdx.x;
    const int bx = key % g.b0, by = (key / g.b0) % g.b1, bz = key / (g.b0 * g.b1);
    const int o0 = bx * BRICK, o1 = by * BRICK, o2 = bz * BRICK;
    for (int e = threadIdx.x; e < REGN; e += ANT) acc[e] = 0ull;
    __syncthreads();
    const uint32_t lo = start[(size_t)key * SUB], hi = start[(size_t)(key + 1) * SUB];
    const int lane = threadIdx.x & 63;
    const int rx = lane % M, ry = (lane >> 4) % M;
    for (uint32_t t = lo + threadIdx.x; t < hi; t += ANT) {
        const int64_t p = idx[t];
        const double x = pos[3 * p], y = pos[3 * p + 1], z = pos[3 * p + 2];
        double wx[M], wy[M], wz[M];
        const int l0 = axis_local<M, PER>(axis_u<PER>(g, 0, x, g.n0), g.n0, o0, wx);
        const int l1 = axis_local<M, PER>(axis_u<PER>(g, 1, y, g.n1), g.n1, o1, wy);
        const int l2 = axis_local<M, PER>(axis_u<PER>(g, 2, z, g.n2), g.n2, o2, wz);
        // rotate the x and y stencil order by lane so that neighbouring lanes
        // (often the same nearest cell) add to different cells in one instruction
        double wxr[M], wyr[M];
        int oxr[M], oyr[M];
#pragma unroll
        for (int c = 0; c < M; ++c) {
            const int sx = c + rx >= M ? c + rx - M : c + rx;
            const int sy = c + ry >= M ? c + ry - M : c + ry;
            wxr[c] = wx[0];
            wyr[c] = wy[0];
#pragma unroll
            for (int q = 1; q < M; ++q) {
                wxr[c] = sx == q ? wx[q] : wxr[c];
                wyr[c] = sy == q ? wy[q] : wyr[c];
            }
            oxr[c] = sx;
            oyr[c] = sy;
        }
#pragma unroll
        for (int a = 0; a < M; ++a) {
#pragma unroll
            for (int b = 0; b < M; ++b) {
                const double wyz = wz[a] * wyr[b] * FIX_ONE;
                const int r = reg_index(l0, l1 + oyr[b], l2 + a);
#pragma unroll
                for (int c = 0; c < M; ++c) {
                    // region: a stencil cell beyond the LDS halo lies outside
                    // the region; its contribution is dropped
                    if (!PER && !(in_reg(l0 + oxr[c]) && in_reg(l1 + oyr[b]) && in_reg(l2 + a))) continue;
                    atomicAdd(&acc[r + oxr[c]], fix_round(wxr[c], wyz));
                }
            }
        }
    }
    __syncthreads();
    unsigned long long* st = stage + (size_t)key * REGN;
    for (int e = threadIdx.x; e < REGN; e += ANT) st[e] = acc[e];
}

// The (brick, brick-local coordinate) pairs along one axis whose LDS region
// entries land on cell i: the cell's own brick, and for the first (last) cell
// of a brick the right (left) halo entry of the previous (next) brick, with
// periodic wrap (a region has no brick before its first or after its last);
// returns how many (1 to 3).
__device__ __forceinline__ int axis_sources(int i, int n, int nbrick, bool periodic, int (&b)[3], int (&l)[3]) {
    const int bi = i / BRICK, li = i - bi * BRICK, w = min(BRICK, n - bi * BRICK);
    int m = 0;
    b[m] = bi;
    l[m++] = li;
    if (li == 0 && (periodic || bi > 0)) {
        const int bp = bi == 0 ? nbrick - 1 : bi - 1;
        b[m] = bp;
        l[m++] = min(BRICK, n - bp * BRICK);
    }
    if (li == w - 1 && (periodic || bi < nbrick - 1)) {
        b[m] = bi == nbrick - 1 ? 0 : bi + 1;
        l[m++] = -1;
    }
    return m;
}

// Every cell: the sum of the staged region entries of the bricks that reach it
// (its own brick's entry, plus halo entries of neighbours for outer-layer
// cells), converted to delta = q * scale - 1.  One block per row
// (blockIdx.x = j, blockIdx.y = k), so the density is written in whole rows.
__global__ void __launch_bounds__(NT) k_gather(AGrid g, bool periodic, const unsigned long long* __restrict__ stage,
                                               double scale, double* __restrict__ d) {
    const int j = blockIdx.x, k = blockIdx.y;
    int b1[3], l1[3], b2[3], l2[3];
    const int m1 = axis_sources(j, g.n1, g.b1, periodic, b1, l1);
    const int m2 = axis_sources(k, g.n2, g.b2, periodic, b2, l2);
    double* row = d + ((int64_t)k * g.n1 + j) * g.n0;
    for (int i = threadIdx.x; i < g.n0; i += NT) {
        int b0[3], l0[3];
        const int m0 = axis_sources(i, g.n0, g.b0, periodic, b0, l0);
        unsigned long long q = 0ull;
        for (int c = 0; c < m2; ++c)
            for (int b = 0; b < m1; ++b)
                for (int a = 0; a < m0; ++a) {
                    const size_t key = ((size_t)b2[c] * g.b1 + b1[b]) * g.b0 + b0[a];
                    q += stage[key * REGN + reg_index(l0[a], l1[b], l2[c])];
                }
        row[i] = (double)q * scale - 1.0;
    }
}

inline int64_t align256(int64_t b) { return (b + 255) & ~(int64_t)255; }

}  // namespace

int64_t mass_assign_bricks(int n0, int n1, int n2) {
    return (int64_t)((n0 + BRICK - 1) / BRICK) * ((n1 + BRICK - 1) / BRICK) * ((n2 + BRICK - 1) / BRICK);
}

int64_t mass_assign_workspace(int64_t np, int n0, int n1, int n2) {
    const int64_t nc = mass_assign_bricks(n0, n1, n2) * SUB;
    return 2 * align256(nc * 4) + align256((nc + 1) * 4) + align256((nc + SCAN_TILE - 1) / SCAN_TILE * 4) +
           2 * align256(np * 4) + align256(mass_assign_bricks(n0, n1, n2) * REGN * 8) +
           align256(mass_assign_bricks(n0, n1, n2) * 4);
}

// Workspace of the allocation-free mass assignment: a file-scope device array
// that every GPU the library runs on holds until the process ends.  Host code
// must not use the array's name as an address (it is a host-side stand-in);
// noalloc_scratch() returns the device address, looked up once per device.
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};
}  // namespace

hipError_t noalloc_scratch(void** ptr) {
    *ptr = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p || reinterpret_cast<uintptr_t>(p) % 256 != 0) return hipErrorInvalidValue;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

hipError_t launch_mass_assign(const double* pos, int64_t np, int n0, int n1, int n2, int scheme, bool periodic,
                              double h, const double* corner, double mean_count, void* work, double* delta,
                              hipStream_t s) {
    AGrid g{n0, n1, n2, (n0 + BRICK - 1) / BRICK, (n1 + BRICK - 1) / BRICK, (n2 + BRICK - 1) / BRICK, h, {0, 0, 0},
            {0, 0, 0}};
    const int nn[3] = {n0, n1, n2};
    if (!periodic)
        for (int a = 0; a < 3; ++a) {
            g.cr[a] = corner[a];
            g.far[a] = nn[a] * h + 2.0 * h;
        }
    const int64_t nb = (int64_t)g.b0 * g.b1 * g.b2, nc = nb * SUB;
    char* w = static_cast<char*>(work);
    uint32_t* count = reinterpret_cast<uint32_t*>(w);
    w += align256(nc * 4);
    uint32_t* cursor = reinterpret_cast<uint32_t*>(w);
    w += align256(nc * 4);
    uint32_t* start = reinterpret_cast<uint32_t*>(w);
    w += align256((nc + 1) * 4);
    uint32_t* sums = reinterpret_cast<uint32_t*>(w);
    const int64_t ntile = (nc + SCAN_TILE - 1) / SCAN_TILE;
    w += align256(ntile * 4);
    uint32_t* keys = reinterpret_cast<uint32_t*>(w);
    w += align256(np * 4);
    uint32_t* idx = reinterpret_cast<uint32_t*>(w);
    w += align256(np * 4);
    unsigned long long* stage = reinterpret_cast<unsigned long long*>(w);
    w += align256(nb * REGN * 8);
    uint32_t* order = reinterpret_cast<uint32_t*>(w);
    const double scale = FIX_INV / mean_count;
    const int chunks = grid_for((np + CHUNK - 1) / CHUNK * NT, 8192);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(nc)), dim3(NT), 0, s, count, nc);
    if (periodic)
        hipLaunchKernelGGL((k_bin<0, true>), dim3(chunks), dim3(NT), 0, s, g, pos, np, count, keys, idx);
    else
        hipLaunchKernelGGL((k_bin<0, false>), dim3(chunks), dim3(NT), 0, s, g, pos, np, count, keys, idx);
    hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)ntile), dim3(NT), 0, s, count, nc, sums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(NT), 0, s, sums, ntile);
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntile), dim3(NT), 0, s, count, nc, sums, start, cursor);
    hipLaunchKernelGGL((k_bin<1, true>), dim3(chunks), dim3(NT), 0, s, g, pos, np, cursor, keys, idx);
    if (scheme == 2)
        hipLaunchKernelGGL(k_brick_order, dim3(1), dim3(ORD_NT), 0, s, start, nb, order);
    else
        order = nullptr;
    if (scheme == 1 && periodic)
        hipLaunchKernelGGL((k_bin_assign<2, true>), dim3((unsigned)nb), dim3(ANT), 0, s, g, pos, start, idx, order, stage);
    else if (scheme == 1)
        hipLaunchKernelGGL((k_bin_assign<2, false>), dim3((unsigned)nb), dim3(ANT), 0, s, g, pos, start, idx, order, stage);
    else if (periodic)
        hipLaunchKernelGGL((k_bin_assign<3, true>), dim3((unsigned)nb), dim3(ANT), 0, s, g, pos, start, idx, order, stage);
    else
        hipLaunchKernelGGL((k_bin_assign<3, false>), dim3((unsigned)nb), dim3(ANT), 0, s, g, pos, start, idx, order, stage);
    hipLaunchKernelGGL(k_gather, dim3(n1, n2), dim3(NT), 0, s, g, periodic, stage, scale, delta);
    return hipGetLastError();
}

}  // namespace vmg
