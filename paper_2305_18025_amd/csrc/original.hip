// The original cubic-scaling bosonic PIMD (appendix "Algorithm Pseudocode",
// the listing of the original method; Background, "cubic scaling bosonic
// PIMD") on the GPU: the comparison path of the quadratic algorithm.
//   1. cycle energies E^[u,v] from their defining sum over the particles
//      u..v of the cycle (Background, the cycle-energy double sum; the bead
//      sum of each particle is formed once);
//   2. the forward recurrence for V^[1,v] (Background), every exponential
//      sum shifted as the appendix "Numerical Stability" describes (its
//      smallest exponent, or the simpler two-candidate shift);
//   3. forces from the derivative of that recurrence, evaluated separately
//      for every bead coordinate b:
//        G_b[v] = sum_{u<=v} W(u,v) (dE^[u,v]/dx_b + G_b[u-1]),  G_b[0] = 0,
//        W(u,v) = exp(-beta (V^[1,u-1] + E^[u,v] - V^[1,v])) / v,
//      and F_b = -G_b[N]: O(N^2) per bead, O(P N^3) in all.
// FP64 throughout.  Kernels run one after the other on the caller's stream
// for one system; the workspace layout is OrigLayout.
#define PIMDB_EXP2_SYM exp2_c_orig
#include "common.h"

namespace pimdb {
namespace {

constexpr int BV = 32;  // v-block of the derivative recurrence
constexpr int SOLVE_T = 256; // threads of the recurrence kernel, one bead coordinate each
constexpr int AST = 66;      // LDS row stride (doubles) of a wave's streamed sums: 64 + 2 against bank conflicts
typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double mi(double d, double box, double ib) {
    return box > 0.0 ? fma(-box, rint(d * ib), d) : d;
}

// coordinate c of bead j (0-based) of particle l (0-based), (P,3,N) layout
__device__ __forceinline__ double bead(const OrigArgs &a, int j, int c, int l) {
    return a.pos[((size_t)j * 3 + c) * a.N + l];
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

__device__ __forceinline__ double readlane_d(double x, int l) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// x of another lane by a DPP move (both 32-bit halves); lanes the row mask
// leaves out get `keep`
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_d(double x, double keep) {
    const long long b = __double_as_longlong(x), k = __double_as_longlong(keep);
    const int lo = __builtin_amdgcn_update_dpp((int)k, (int)b, CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(k >> 32), (int)(b >> 32), CTRL, ROWS, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Whole-wave sum or minimum through DPP lane moves (the wave must be fully
// active): lane pairs and quads, half-row and row mirrors give every lane
// its row's result; two row broadcasts carry rows 0..2 into row 3; lane 63
// holds the result, which every lane receives.
template <bool MIN>
__device__ __forceinline__ double wave_reduce_dpp(double x) {
    const double id = MIN ? INFINITY : 0.0;
    auto op = [](double p, double q) { return MIN ? fmin(p, q) : p + q; };
    x = op(x, dpp_d<0xB1, 0xf>(x, id)); // quad_perm [1,0,3,2]
    x = op(x, dpp_d<0x4E, 0xf>(x, id)); // quad_perm [2,3,0,1]
    x = op(x, dpp_d<0x141, 0xf>(x, id)); // row_half_mirror
    x = op(x, dpp_d<0x140, 0xf>(x, id)); // row_mirror
    x = op(x, dpp_d<0x142, 0xa>(x, id)); // row_bcast:15 into rows 1 and 3
    x = op(x, dpp_d<0x143, 0xc>(x, id)); // row_bcast:31 into rows 2 and 3
    return readlane_d(x, 63);
}

// Per particle: the interior spring sum sum_j |r^{j+1} - r^j|^2 and the
// link |r_{l+1}^1 - r_l^P|^2 (0 for the last particle), both without k.
__global__ void k_orig_springs(OrigArgs a) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= a.N) return;
    const double box = a.box, ib = a.inv_box;
    double px = bead(a, 0, 0, l), py = bead(a, 0, 1, l), pz = bead(a, 0, 2, l);
    bool bad = !(isfinite(px) && isfinite(py) && isfinite(pz));
    double s = 0.0;
    for (int j = 1; j < a.P; ++j) {
        const double qx = bead(a, j, 0, l), qy = bead(a, j, 1, l), qz = bead(a, j, 2, l);
        bad |= !(isfinite(qx) && isfinite(qy) && isfinite(qz));
        const double dx = mi(qx - px, box, ib), dy = mi(qy - py, box, ib), dz = mi(qz - pz, box, ib);
        s += dx * dx + dy * dy + dz * dz;
        px = qx;
        py = qy;
        pz = qz;
    }
    a.ws[OrigLayout::ein(a.N) + l] = s;
    double lk = 0.0;
    if (l + 1 < a.N) {
        const double dx = mi(bead(a, 0, 0, l + 1) - px, box, ib);
        const double dy = mi(bead(a, 0, 1, l + 1) - py, box, ib);
        const double dz = mi(bead(a, 0, 2, l + 1) - pz, box, ib);
        lk = dx * dx + dy * dy + dz * dz;
    }
    a.ws[OrigLayout::lnk(a.N) + l] = lk;
    if (bad) set_flag(a.flags, ST_NONFINITE_IN);
}

// E^[u,v] = k (sum_{l=u}^{v} interior(l) + sum_{l=u}^{v-1} link(l)
//             + |r_u^1 - r_v^P|^2), one thread per (u, v); 0 for u > v.
__global__ void k_orig_cycle(OrigArgs a) {
    const int N = a.N;
    const int u = blockIdx.x * blockDim.x + threadIdx.x; // 0-based
    const int v = blockIdx.y;                            // 0-based
    if (u >= N) return;
    double e = 0.0;
    if (u <= v) {
        const double *ein = a.ws + OrigLayout::ein(N), *lnk = a.ws + OrigLayout::lnk(N);
        double s = 0.0;
        for (int l = u; l <= v; ++l) s += ein[l];
        for (int l = u; l < v; ++l) s += lnk[l];
        const double box = a.box, ib = a.inv_box;
        const double dx = mi(bead(a, 0, 0, u) - bead(a, a.P - 1, 0, v), box, ib);
        const double dy = mi(bead(a, 0, 1, u) - bead(a, a.P - 1, 1, v), box, ib);
        const double dz = mi(bead(a, 0, 2, u) - bead(a, a.P - 1, 2, v), box, ib);
        e = a.k * (s + dx * dx + dy * dy + dz * dz);
    }
    a.ws[OrigLayout::Et(N) + (size_t)v * N + u] = e;
}

// Er = the transpose of Et, in 32 x 32 tiles.
__global__ void k_orig_transpose(OrigArgs a) {
    __shared__ double tile[32][33];
    const int N = a.N;
    const int u0 = blockIdx.x * 32, v0 = blockIdx.y * 32;
    const double *Et = a.ws + OrigLayout::Et(N);
    double *Er = a.ws + OrigLayout::Er(N);
    const int tx = threadIdx.x, ty = threadIdx.y;
    for (int r = ty; r < 32; r += 8) {
        const int v = v0 + r, u = u0 + tx;
        tile[r][tx] = (v < N && u < N) ? Et[(size_t)v * N + u] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int u = u0 + r, v = v0 + tx;
        if (u < N && v < N) Er[(size_t)u * N + v] = tile[tx][r];
    }
}

// exp(-beta V^[1,v]) = (1/v) sum_{u=1}^{v} exp(-beta (V^[1,u-1] + E^[u,v])),
// V^[1,0] = 0, then the energy V^[1,N] plus the trap's scaled potential.
// Steps v in blocks of FB: the terms u <= v0 of the block's steps (V known)
// are summed first by all four waves, each over a quarter of u, relative
// to their own smallest exponent; then wave 0 steps through the block, lane
// i holding V^[1,v0+i] and the term of u = v0+1+i, with the block's cycle
// energies staged in LDS while the partial sums run.  Each step's shift is
// the smallest exponent over all its terms (or the two-candidate shift),
// and the partial sums are rescaled to it.
constexpr int FB = 63; // steps per block; lane 63 carries the partial sums

__global__ void __launch_bounds__(256) k_orig_forward(OrigArgs a) {
    extern __shared__ double Vs[]; // N + 1
    __shared__ double pm[4][64], ps[4][64];
    __shared__ double tri[FB][FB + 1], e1[FB]; // [i][j] = E^[v0+1+j, v0+1+i]; E^[1, v0+1+i]
    const int N = a.N, t = threadIdx.x, lane = t & 63, w = t >> 6;
    const double *Et = a.ws + OrigLayout::Et(N), *Er = a.ws + OrigLayout::Er(N);
    const double beta = a.beta;
    if (t == 0) Vs[0] = 0.0;
    __syncthreads();
    for (int v0 = 0; v0 < N; v0 += FB) {
        for (int e = t; e < FB * FB; e += 256) {
            const int i = e / FB, jj = e - i * FB;
            tri[i][jj] = (v0 + i < N && v0 + jj < N) ? Et[(size_t)(v0 + i) * N + v0 + jj] : 0.0;
        }
        if (t < FB) e1[t] = v0 + t < N ? Et[(size_t)(v0 + t) * N] : 0.0;
        if (lane < FB) {
            const int v = v0 + 1 + lane;
            const int ua = 1 + (int)(((int64_t)v0 * w) / 4), ub = (int)(((int64_t)v0 * (w + 1)) / 4);
            // one pass: the sum relative to the smallest exponent so far,
            // rescaled when a smaller one comes (one exponential per term)
            double m = INFINITY, s = 0.0;
            if (v <= N) {
                for (int u0 = ua; u0 <= ub; u0 += 8) {
                    double xv[8];
#pragma unroll
                    for (int r = 0; r < 8; ++r)
                        xv[r] = u0 + r <= ub ? Vs[u0 + r - 1] + Er[(size_t)(u0 + r - 1) * N + (v - 1)] : INFINITY;
#pragma unroll
                    for (int r = 0; r < 8; ++r) {
                        if (xv[r] < INFINITY) {
                            const double d = xv[r] - m; // -inf before the first term
                            const double e = exp(-beta * fabs(d));
                            if (d < 0.0) {
                                s = s * e + 1.0;
                                m = xv[r];
                            } else {
                                s += e;
                            }
                        }
                    }
                }
            }
            pm[w][lane] = m;
            ps[w][lane] = s;
        } else {
            pm[w][lane] = INFINITY;
            ps[w][lane] = 0.0;
        }
        __syncthreads();
        if (w == 0) {
            double mp = fmin(fmin(pm[0][lane], pm[1][lane]), fmin(pm[2][lane], pm[3][lane]));
            double sp = 0.0;
            if (mp < INFINITY) {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (pm[q][lane] < INFINITY) sp += ps[q][lane] * exp(-beta * (pm[q][lane] - mp));
            }
            double myV = Vs[v0]; // lane i < FB: V^[1,v0+i] once known (lane 0 now)
            const int nv = min(FB, N - v0);
            const double lnv = log((double)(v0 + 1 + lane)); // lane i: ln(v) of step i
            const double ib = 1.0 / beta;
            for (int i = 0; i < nv; ++i) {
                const int v = v0 + 1 + i;
                // lanes u - v0 - 1 <= i hold the new terms; lane FB the partial sums
                const bool act = lane <= i;
                const double mpv = readlane_d(mp, i), spv = readlane_d(sp, i);
                double x = act ? myV + tri[i][min(lane, FB - 1)] : INFINITY; // V^[1,u-1] + E^[u,v]
                if (lane == FB) x = mpv;
                double sh;
                if (a.two_term)
                    sh = fmin(e1[i], readlane_d(x, i)); // E^[1,v] and V^[1,v-1] + E^[v,v]
                else
                    sh = wave_reduce_dpp<true>(x);
                const double ex = x < INFINITY ? exp(-beta * (x - sh)) : 0.0;
                const double s = wave_reduce_dpp<false>(lane == FB ? spv * ex : ex);
                const double Vv = sh - (log(s) - readlane_d(lnv, i)) * ib;
                if (lane == i + 1) myV = Vv;
                if (lane == 0) Vs[v] = Vv;
            }
        }
        __syncthreads();
    }
    double *Vg = a.ws + OrigLayout::V(N);
    for (int v = t; v <= N; v += 256) Vg[v] = Vs[v];
    double et = 0.0;
    if (a.trapc != 0.0) {
        const size_t n = (size_t)3 * a.P * N;
        for (size_t i = t; i < n; i += 256) et += a.pos[i] * a.pos[i];
        et = wave_sum(et);
        if (lane == 0) pm[w][0] = et;
        __syncthreads();
        et = 0.5 * a.trapc * (pm[0][0] + pm[1][0] + pm[2][0] + pm[3][0]);
    }
    if (t == 0) {
        const double V = Vs[N] + et;
        if (!isfinite(V)) set_flag(a.flags, ST_NONFINITE_OUT);
        if (a.energy) *a.energy = V;
    }
}

// W[g][v-1] = exp(-beta (V^[1,g] + E^[g+1,v] - V^[1,v])) / v for g < v, else 0.
__global__ void k_orig_weights(OrigArgs a) {
    const int N = a.N;
    const int vv = blockIdx.x * blockDim.x + threadIdx.x, g = blockIdx.y; // column v-1, row g
    if (vv >= N) return;
    const double *Er = a.ws + OrigLayout::Er(N), *V = a.ws + OrigLayout::V(N);
    double w = 0.0;
    if (g <= vv) w = exp(-a.beta * (V[g] + Er[(size_t)g * N + vv] - V[vv + 1])) / (double)(vv + 1);
    a.ws[OrigLayout::W(N) + (size_t)g * N + vv] = w;
}

// Column prefix sums C[L][v-1] = sum_{g<L} W[g][v-1], and for particle l
// (= v) the last bead's derivative sum at v = l, where the cycle [u, l]
// closes on bead 1 of u:
//   T[l] = sum_{u<=l} W(u,l) ((r_l^P - r_l^{P-1}) + (r_l^P - r_u^1)).
__global__ void k_orig_prefix(OrigArgs a) {
    const int N = a.N, P = a.P;
    const int vv = blockIdx.x * blockDim.x + threadIdx.x;
    if (vv >= N) return;
    const double *W = a.ws + OrigLayout::W(N);
    double *C = a.ws + OrigLayout::C(N), *T = a.ws + OrigLayout::T(N);
    double c = 0.0;
    C[vv] = 0.0;
    for (int g0 = 0; g0 < N; g0 += 16) { // loads first, then the running sum
        double wv[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) wv[r] = g0 + r < N ? W[(size_t)(g0 + r) * N + vv] : 0.0;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            if (g0 + r < N) {
                c += wv[r];
                C[(size_t)(g0 + r + 1) * N + vv] = c;
            }
        }
    }
    const int l = vv;
    const double box = a.box, ib = a.inv_box;
    double xl[3], in[3], t3[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
        xl[cc] = bead(a, P - 1, cc, l);
        in[cc] = mi(xl[cc] - bead(a, P - 2, cc, l), box, ib);
    }
    for (int u0 = 0; u0 <= l; u0 += 8) {
        double wv[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) wv[r] = u0 + r <= l ? W[(size_t)(u0 + r) * N + l] : 0.0;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            if (u0 + r <= l) {
#pragma unroll
                for (int cc = 0; cc < 3; ++cc)
                    t3[cc] += wv[r] * (in[cc] + mi(xl[cc] - bead(a, 0, cc, u0 + r), box, ib));
            }
        }
    }
    T[3 * l] = t3[0];
    T[3 * l + 1] = t3[1];
    T[3 * l + 2] = t3[2];
}

// The derivative recurrence, one thread per bead coordinate b = (l, j, c)
// (particle-major, so a workgroup covers two to four particles).  G_b[v] = 0
// for v < l: cycles [u, v] with v < l do not contain particle l.  For
// v >= l the terms with u <= l (cycles that contain l) have G_b[u-1] = 0 and
// a derivative dE^[u,v]/dx_b that takes one value for u < l (cA) and one
// for u = l (cB, plus for bead 1 the closing spring to bead P of v), so
// their sum is cA C[l-1][v-1] + cB W[l-1][v-1]; the last bead at v = l
// (closing spring to bead 1 of u) is the sum T.  The rest, the terms
// u-1 = g >= l, is a lower-triangular recurrence over g in blocks of BV
// values of v: the terms of earlier blocks' G values form a dense product
// (a tile of W^T in LDS times the wave's G values) on the FP64 matrix
// cores; the block's own triangle follows, one lane per right-hand side.
__global__ void __launch_bounds__(SOLVE_T) k_orig_solve(OrigArgs a) {
    const int N = a.N, P = a.P, t = threadIdx.x;
    const int64_t NB = (int64_t)3 * P * N;
    const int64_t b = (int64_t)blockIdx.x * SOLVE_T + t;
    const bool live = b < NB;
    const int64_t bb = live ? b : NB - 1;
    const int lz = (int)(bb / (3 * P)); // particle, 0-based
    const int rem = (int)(bb - (int64_t)lz * 3 * P);
    const int j = rem / 3, c = rem - 3 * j;
    const int l1 = lz + 1; // particle, 1-based
    const int lmin1 = (int)(((int64_t)blockIdx.x * SOLVE_T) / (3 * P)) + 1;
    const double *W = a.ws + OrigLayout::W(N), *C = a.ws + OrigLayout::C(N), *T = a.ws + OrigLayout::T(N);
    // this workgroup's history: [v-1][t], SOLVE_T per row
    double *G = a.ws + OrigLayout::G(N) + (size_t)blockIdx.x * N * SOLVE_T;
    __shared__ double tile[BV][BV + 1]; // W[g][v-1], g in the chunk, v in the block
    __shared__ double dt[BV][BV];       // W[g][v-1], g and v in the block
    __shared__ double accs[SOLVE_T / 64 * BV * AST]; // each wave's streamed sums, [v][b]
    const int w = t >> 6, lane = t & 63, li = lane & 15, lk = lane >> 4;
    int lb[4]; // particles (1-based) of this lane's B columns
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int64_t bq = (int64_t)blockIdx.x * SOLVE_T + 64 * w + 16 * nt + li;
        lb[nt] = (int)((bq < NB ? bq : NB - 1) / (3 * P)) + 1;
    }
    const double box = a.box, ib = a.inv_box, mw2 = a.mw2;
    // dE/dx_b = m w^2 ((x - prev) + (x - next)) for the cycles that contain l
    const double x0 = bead(a, j, c, lz);
    int kind; // 0 interior bead, 1 bead 1, 2 bead P
    double cA, cB;
    if (j == 0) {
        kind = 1;
        cB = mw2 * mi(x0 - bead(a, 1, c, lz), box, ib);
        cA = lz > 0 ? cB + mw2 * mi(x0 - bead(a, P - 1, c, lz - 1), box, ib) : cB;
    } else if (j == P - 1) {
        kind = 2;
        cB = mw2 * mi(x0 - bead(a, P - 2, c, lz), box, ib);
        if (l1 < N) cB += mw2 * mi(x0 - bead(a, 0, c, lz + 1), box, ib);
        cA = cB;
    } else {
        kind = 0;
        cB = mw2 * (mi(x0 - bead(a, j + 1, c, lz), box, ib) + mi(x0 - bead(a, j - 1, c, lz), box, ib));
        cA = cB;
    }
    const double *Wl = W + (size_t)lz * N; // W[l-1][v-1]
    const double *Cl = C + (size_t)lz * N; // C[l-1][v-1]
    double last = 0.0;
    for (int v0 = ((lmin1 - 1) / BV) * BV + 1; v0 <= N; v0 += BV) {
        // rows g in [lmin1, v0) in chunks of BV on the matrix cores: for this
        // wave's 64 right-hand sides (4 column tiles of 16) and the block's
        // 32 values of v (2 row tiles), D[v][b] += W^T[v][g] G[g][b], 4 g per
        // v_mfma_f64_16x16x4f64 (A: lane l holds A[l%16][l/16]; B: lane l
        // holds B[l/16][l%16]; D: lane l, element r holds D[4r + l/16][l%16])
        d4 D[2][4];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) D[mt][nt] = d4{0.0, 0.0, 0.0, 0.0};
        for (int gc = lmin1; gc < v0; gc += BV) {
            // this lane's B values of the chunk (rows before the column's
            // particle, or past the chunk, read row 1 and count zero), loaded
            // while the W tile is staged
            double bv[BV / 4][4];
#pragma unroll
            for (int kk = 0; kk < BV / 4; ++kk) {
                const int g = gc + 4 * kk + lk;
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    const bool use = g < v0 && g >= lb[nt];
                    const double x = G[(size_t)((use ? g : 1) - 1) * SOLVE_T + 64 * w + 16 * nt + li];
                    bv[kk][nt] = use ? x : 0.0;
                }
            }
            __syncthreads();
            for (int e = t; e < BV * BV; e += SOLVE_T) {
                const int r = e / BV, i = e - r * BV;
                const int g = gc + r, v = v0 + i;
                tile[r][i] = (g < v0 && v <= N) ? W[(size_t)g * N + (v - 1)] : 0.0;
            }
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < BV / 4; ++kk) {
                double av[2];
#pragma unroll
                for (int mt = 0; mt < 2; ++mt) av[mt] = tile[4 * kk + lk][16 * mt + li];
#pragma unroll
                for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt)
                        D[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[mt], bv[kk][nt], D[mt][nt], 0, 0, 0);
            }
        }
        // to one lane per right-hand side, through this wave's LDS rows
        double *aw = accs + (size_t)w * BV * AST;
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                for (int r = 0; r < 4; ++r) aw[(16 * mt + 4 * r + lk) * AST + 16 * nt + li] = D[mt][nt][r];
        double acc[BV];
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int i = 0; i < BV; ++i) acc[i] = aw[i * AST + lane];
        __syncthreads();
        for (int e = t; e < BV * BV; e += SOLVE_T) {
            const int r = e / BV, i = e - r * BV;
            const int g = v0 + r, v = v0 + i;
            dt[r][i] = (r < i && v <= N) ? W[(size_t)g * N + (v - 1)] : 0.0;
        }
        __syncthreads();
        // the block's own triangle: g = v0 + i feeds v0 + i2 for i2 > i
#pragma unroll
        for (int i = 0; i < BV; ++i) {
            const int v = v0 + i;
            if (v <= N && v >= l1) {
                double gv;
                if (kind == 2 && v == l1) {
                    gv = mw2 * T[3 * lz + c];
                } else {
                    const double wl = Wl[v - 1];
                    gv = acc[i] + cA * Cl[v - 1] + cB * wl;
                    if (kind == 1) gv += mw2 * wl * mi(x0 - bead(a, P - 1, c, v - 1), box, ib);
                }
                G[(size_t)(v - 1) * SOLVE_T + t] = gv;
#pragma unroll
                for (int i2 = i + 1; i2 < BV; ++i2) acc[i2] = fma(dt[i][i2], gv, acc[i2]);
                last = gv;
            }
        }
    }
    if (live && a.out) {
        const double f = -last - a.trapc * x0;
        a.out[((size_t)j * 3 + c) * N + lz] = f;
        if (!isfinite(f)) set_flag(a.flags, ST_NONFINITE_OUT);
    }
}

} // namespace

hipError_t launch_original(const OrigArgs &a, hipStream_t st) {
    const int N = a.N;
    hipLaunchKernelGGL(k_orig_springs, dim3((N + 255) / 256), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_orig_cycle, dim3((N + 63) / 64, N), dim3(64), 0, st, a);
    hipLaunchKernelGGL(k_orig_transpose, dim3((N + 31) / 32, (N + 31) / 32), dim3(32, 8), 0, st, a);
    hipLaunchKernelGGL(k_orig_forward, dim3(1), dim3(256), (size_t)(N + 1) * sizeof(double), st, a);
    if (a.out) {
        hipLaunchKernelGGL(k_orig_weights, dim3((N + 255) / 256, N), dim3(256), 0, st, a);
        hipLaunchKernelGGL(k_orig_prefix, dim3((N + 255) / 256), dim3(256), 0, st, a);
        const int64_t NB = (int64_t)3 * a.P * N;
        hipLaunchKernelGGL(k_orig_solve, dim3((unsigned)((NB + SOLVE_T - 1) / SOLVE_T)), dim3(SOLVE_T), 0, st, a);
    }
    return hipGetLastError();
}

} // namespace pimdb
