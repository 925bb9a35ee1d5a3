// Mass assignment: unit-mass particles to the density contrast on a periodic
// mesh (Sec. VI: the mesh density comes from triangular-shaped-cloud
// assignment of the particles; cloud in cell is the next-lower-order member of
// the same family of shape functions).
//
// Accumulation is in 64-bit fixed point (2^-40 of a particle's mass per unit):
// every contribution is rounded once, then added with an integer atomic, so the
// sums do not depend on the order in which the atomics land and the result is
// bitwise reproducible.  The density buffer itself holds the integers until the
// finishing pass converts them in place to delta.
#include "device_common.h"
#include "vmg_internal.h"

namespace vmg {
namespace {

constexpr double FIX_ONE = 1099511627776.0;           // 2^40
constexpr double FIX_INV = 1.0 / 1099511627776.0;     // 2^-40

__global__ void __launch_bounds__(NT) k_zero_u64(unsigned long long* __restrict__ q, int64_t N) {
    for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < N; e += (int64_t)gridDim.x * NT) q[e] = 0ull;
}

// Cell index i in [-n, 3n) wrapped onto [0, n).
__device__ __forceinline__ int wrap3(int i, int n) {
    i += i < 0 ? n : 0;
    i -= i >= n ? n : 0;
    i -= i >= n ? n : 0;
    return i;
}

// Per-axis cells and weights of one coordinate x (box units) on n cells.
// CIC: u' = u - 1/2, weights (1 - t, t) on cells floor(u'), floor(u') + 1.
// TSC: nearest cell c, d = u - (c + 1/2), weights (1/2 - d)^2/2, 3/4 - d^2,
// (1/2 + d)^2/2 on cells c - 1, c, c + 1.
template <int M>
__device__ __forceinline__ void axis_weights(double x, int n, int (&c)[M], double (&w)[M]) {
    const double u = (x - floor(x)) * (double)n;       // [0, n]
    if constexpr (M == 2) {
        const double f = floor(u - 0.5);
        const double t = (u - 0.5) - f;
        c[0] = wrap3((int)f, n);
        c[1] = wrap3((int)f + 1, n);
        w[0] = 1.0 - t;
        w[1] = t;
    } else {
        const double f = floor(u);
        const double d = u - (f + 0.5);
        c[0] = wrap3((int)f - 1, n);
        c[1] = wrap3((int)f, n);
        c[2] = wrap3((int)f + 1, n);
        const double a = 0.5 - d, b = 0.5 + d;
        w[0] = 0.5 * (a * a);
        w[1] = 0.75 - d * d;
        w[2] = 0.5 * (b * b);
    }
}

// One particle per thread (grid-stride).  The y-z weights are folded into the
// x weights before rounding, so each of the M^3 contributions is rounded once.
template <int M>
__global__ void __launch_bounds__(NT) k_assign(const double* __restrict__ pos, int64_t np, int n0, int n1, int n2,
                                               unsigned long long* __restrict__ q) {
    for (int64_t p = (int64_t)blockIdx.x * NT + threadIdx.x; p < np; p += (int64_t)gridDim.x * NT) {
        const double x = pos[3 * p], y = pos[3 * p + 1], z = pos[3 * p + 2];
        if (!isfinite(x) || !isfinite(y) || !isfinite(z)) continue;
        int cx[M], cy[M], cz[M];
        double wx[M], wy[M], wz[M];
        axis_weights<M>(x, n0, cx, wx);
        axis_weights<M>(y, n1, cy, wy);
        axis_weights<M>(z, n2, cz, wz);
#pragma unroll
        for (int a = 0; a < M; ++a) {
#pragma unroll
            for (int b = 0; b < M; ++b) {
                const double wyz = wz[a] * wy[b] * FIX_ONE;
                unsigned long long* row = q + ((int64_t)cz[a] * n1 + cy[b]) * n0;
#pragma unroll
                for (int c = 0; c < M; ++c)
                    atomicAdd(row + cx[c], (unsigned long long)__double2ll_rn(wx[c] * wyz));
            }
        }
    }
}

// In place: integer mass q (units of 2^-40) -> delta = q * scale - 1.
__global__ void __launch_bounds__(NT) k_assign_finish(double* __restrict__ d, int64_t N, double scale) {
    unsigned long long* q = reinterpret_cast<unsigned long long*>(d);
    for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < N; e += (int64_t)gridDim.x * NT)
        d[e] = (double)q[e] * scale - 1.0;
}

}  // namespace

hipError_t launch_mass_assign(const double* pos, int64_t np, int n0, int n1, int n2, int scheme, double* delta,
                              hipStream_t s) {
    const int64_t N = (int64_t)n0 * n1 * n2;
    unsigned long long* q = reinterpret_cast<unsigned long long*>(delta);
    hipLaunchKernelGGL(k_zero_u64, dim3(grid_for(N)), dim3(NT), 0, s, q, N);
    if (scheme == 1)
        hipLaunchKernelGGL(k_assign<2>, dim3(grid_for(np)), dim3(NT), 0, s, pos, np, n0, n1, n2, q);
    else
        hipLaunchKernelGGL(k_assign<3>, dim3(grid_for(np)), dim3(NT), 0, s, pos, np, n0, n1, n2, q);
    hipLaunchKernelGGL(k_assign_finish, dim3(grid_for(N)), dim3(NT), 0, s, delta, N,
                       FIX_INV * ((double)N / (double)np));
    return hipGetLastError();
}

}  // namespace vmg
