// Scaled pair interaction (Theory, the bosonic partition function: the
// interaction of every imaginary-time slice scaled by 1/P)
//   U-bar = (1/P) sum_j sum_{a<b} U(|r_a^j - r_b^j|),
// with the caller's Gaussian U(r) = g exp(-r^2 / (2 sigma^2)), and its forces
//   F_a^j = (1/P) sum_{b != a} (g / sigma^2) exp(-r_ab^2 / (2 sigma^2)) (r_a^j - r_b^j).
// O(P N^2) pairs, each computed in FP64 from the minimum-image displacement:
// a workgroup takes iblock particles of one slice and streams the slice's
// particles through LDS in tiles; every pair's exponential is 2^x from the
// library's minimax polynomial.  Partial energies go to one slot per
// workgroup and a second launch sums each system's slots in a fixed order
// (the same result on every run).
#define PIMDB_EXP2_SYM exp2_c_pair
#include "common.h"

namespace pimdb {
namespace {

constexpr int PT = 256; // partner particles per LDS tile

template <bool BOX>
__global__ void __launch_bounds__(256) k_pair(PairArgs a) {
    __shared__ double tx[PT], ty[PT], tz[PT];
    __shared__ double red[256];
    const PairItem it = a.items[blockIdx.x];
    const SysDesc sd = a.sys[it.sys];
    const int N = sd.N, P = sd.P, t = threadIdx.x, T = blockDim.x;
    const int64_t off = a.offs ? a.offs[it.sys] : sd.off;
    if (off < 0) return; // a skipped system of the caller-packed batch
    const size_t NN = (size_t)N;
    const double *X = a.pos + off + (size_t)it.j * 3 * NN; // slice j: x[N], y[N], z[N]
    const int i = it.i0 + t;
    const bool live = i < N;
    const double xi = live ? X[i] : 0.0, yi = live ? X[NN + i] : 0.0, zi = live ? X[2 * NN + i] : 0.0;
    const double box = a.box, ib = a.inv_box, c2 = a.c2;
    double fx = 0.0, fy = 0.0, fz = 0.0, e = 0.0;
    for (int k0 = 0; k0 < N; k0 += PT) {
        __syncthreads();
        for (int q = t; q < PT; q += T) {
            const int k = k0 + q;
            tx[q] = k < N ? X[k] : 0.0;
            ty[q] = k < N ? X[NN + k] : 0.0;
            tz[q] = k < N ? X[2 * NN + k] : 0.0;
        }
        __syncthreads();
        const int nk = min(PT, N - k0);
        for (int q = 0; q < nk; ++q) {
            const double dx = mimg<BOX>(xi - tx[q], box, ib);
            const double dy = mimg<BOX>(yi - ty[q], box, ib);
            const double dz = mimg<BOX>(zi - tz[q], box, ib);
            const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
            double p;
            int n;
            exp2x(fmax(c2 * r2, -2100.0), p, n); // below -1075 the term is 0
            const double u = (k0 + q == i) ? 0.0 : ldexp(p, n);
            e += u;
            fx = fma(u, dx, fx);
            fy = fma(u, dy, fy);
            fz = fma(u, dz, fz);
        }
    }
    const double inv_p = 1.0 / (double)P;
    if (live && a.out) {
        const double sc = a.sign * a.g * a.inv_s2 * inv_p * (a.gscale ? a.gscale[it.sys] : 1.0);
        double *o = a.out + off + (size_t)it.j * 3 * NN + i;
        const double ox = sc * fx + (a.accumulate ? o[0] : 0.0);
        const double oy = sc * fy + (a.accumulate ? o[NN] : 0.0);
        const double oz = sc * fz + (a.accumulate ? o[2 * NN] : 0.0);
        o[0] = ox;
        o[NN] = oy;
        o[2 * NN] = oz;
        if (!(isfinite(ox) && isfinite(oy) && isfinite(oz))) set_flag(a.flags, ST_NONFINITE_OUT);
    }
    if (a.energy) {
        const double s = block_sum(live ? e : 0.0, red);
        if (t == 0) a.epart[blockIdx.x] = 0.5 * a.g * inv_p * s; // each pair met twice
    }
}

// Energy of each system: its items' partials in item order.
__global__ void __launch_bounds__(64) k_pair_energy(PairArgs a) {
    const int s = blockIdx.x, t = threadIdx.x;
    if (a.offs && a.offs[s] < 0) return; // skipped: its energy is not written
    const int b0 = a.beg[s], b1 = a.beg[s + 1];
    double v = 0.0;
    for (int b = b0 + t; b < b1; b += 64) v += a.epart[b];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (t == 0) {
        const double E = a.accumulate ? a.energy[s] + v : v;
        if (!isfinite(E)) set_flag(a.flags, ST_NONFINITE_OUT);
        a.energy[s] = E;
    }
}

} // namespace

hipError_t launch_pair(const PairArgs &a, int nitems, int S, hipStream_t st) {
    if (nitems <= 0) return hipSuccess;
    if (a.box > 0)
        hipLaunchKernelGGL(k_pair<true>, dim3(nitems), dim3(a.iblock), 0, st, a);
    else
        hipLaunchKernelGGL(k_pair<false>, dim3(nitems), dim3(a.iblock), 0, st, a);
    if (a.energy) hipLaunchKernelGGL(k_pair_energy, dim3(S), dim3(64), 0, st, a);
    return hipGetLastError();
}

} // namespace pimdb
