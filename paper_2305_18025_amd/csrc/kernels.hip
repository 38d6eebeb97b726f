// HIP kernels for gfx950: bosonic exchange potential V^[1,N] and bead forces.
//
// Method (Feldman & Hirshberg, "Quadratic Scaling Bosonic PIMD"):
//   cycle energies E^[u,v]                      Theory, "Reducing the potential"
//   forward  exp(-b V^[1,v]) = (1/v) sum_u exp(-b(V^[1,u-1] + E^[u,v]))
//                                               Background, recurrence for V^[1,N]
//   backward exp(-b V^[u,N]) = sum_l (1/l) exp(-b(E^[u,l] + V^[l+1,N]))
//                                               Theory, "Connection probabilities"
//   Pr[l -> l+1] = 1 - exp(-b(V^[1,l] + V^[l+1,N] - V^[1,N]))
//   Pr[l -> u]   = (1/l) exp(-b(V^[1,u-1] + E^[u,l] + V^[l+1,N] - V^[1,N])), u <= l
//                                               Methods, "Expressions for connection probabilities"
//   exterior forces = Pr-weighted spring forces Theory, "Force on exterior beads"
//
// How this implementation evaluates it (every step is exact algebra on the
// definitions above; only rounding differs):
//
// 1. Open-chain gauge.  For any constants c_l, replacing E^[u,v] by
//    E^[u,v] - sum_{l=u}^{v} c_l and V^[1,v] by V^[1,v] - sum_{l<=v} c_l (and
//    V^[u,N] by V^[u,N] - sum_{l>=u} c_l) leaves both recursions and every
//    probability exponent unchanged.  With c_l = E_int(l) + lambda_l,
//    lambda_l = s(l, l+1) for l < N and lambda_N = s(N, N), where
//    s(a, b) = k |r_a^P - r_b^1|^2, the reduced cycle energy is simply
//        Etilde[u,v] = s(v, u) - lambda_v,
//    so the O(N^2) part needs only the 2N endpoint beads and no prefix sums;
//    the interior springs enter only the energy, as the constant sum_l c_l.
// 2. Extended-exponent numbers.  The recursions carry Z = exp(-b Vtilde) as a
//    double mantissa times 2^(int exponent), so no log or exp of a potential
//    is ever needed and no magnitude is lost to the size of V.  Each term
//    K(u,v) = exp(-b Etilde[u,v]) = 2^x is formed as mantissa 2^frac(x)
//    (own polynomial) times 2^round(x).
// 3. Right-looking recursions.  Thread-owned accumulators: when Z_f[u-1] is
//    known, every accumulator v >= u adds Z_f[u-1] K(u,v) at once, and the
//    owner of v = u then holds Z_f[u] = acc/u.  One workgroup barrier per
//    step; the only serial chain is the owner's multiply-add and rescale.
//    The backward recursion is the same with rows and columns exchanged.
//    Forward and backward run concurrently in separate workgroups.
// 4. Forces without materialised probabilities.  Pr[v -> u] (u <= v) is the
//    forward term of accumulator v divided by its sum, times
//    rho_v = Z_f[v] Z_b[v+1] / Z_f[N] = 1 - Pr[v -> v+1]; likewise the column
//    Pr[l -> u] (l >= u) is the backward term of accumulator u over its sum,
//    times rho_{u-1}.  Accumulating the term-weighted endpoint displacements
//    next to the sums therefore gives sum_u Pr[v -> u] (r_v^P - r_u^1) and
//    sum_l Pr[l -> u] (r_l^P - r_u^1) directly: the exterior-bead forces cost
//    O(N) after the recursions instead of a third O(N^2) pass.
//
// Layout: positions/forces (P, 3, N) per system, bead-major SoA, packed.

#include "internal.h"

#include <hip/hip_runtime.h>
#include <math.h>

namespace pimdb {

constexpr int CH = 512;                  // particles staged in LDS per chunk
constexpr double LN2 = 0.6931471805599453;
constexpr double XLO = -536870912.0;     // -2^29: lower clamp of a term exponent
constexpr double XHI = 268435456.0;      //  2^28: bound on h = -kappa |d_ref|^2
constexpr int EMIN = -(1 << 30);         // exponent of an empty accumulator

enum StatusBits { ST_NONFINITE_IN = 1, ST_NONFINITE_OUT = 2, ST_RANGE = 4 };

// 2^f for |f| <= 1/2: degree-11 minimax polynomial (relative approximation
// error 3e-18, below the rounding of its evaluation; coefficients from
// gen_exp2_coeffs.py), highest degree first.  Kept in constant memory so the
// wave-uniform coefficients live in scalar registers and every Horner step
// is one v_fma_f64.
__constant__ double EXP2_C[12] = {
    4.4352809446103363e-10, 7.074105626245659e-09, 1.0178198033328528e-07, 1.321543308959463e-06,
    1.5252733489960805e-05, 0.00015403530462514614, 0.001333355814678995, 0.009618129107588335,
    0.055504108664819925,   0.24022650695910155,    0.6931471805599453,    1.0};

__device__ __forceinline__ double exp2_frac(double f) {
    double p = EXP2_C[0];
#pragma unroll
    for (int i = 1; i < 12; ++i) p = fma(p, f, EXP2_C[i]);
    return p;
}

template <bool BOX>
__device__ __forceinline__ double mimg(double d, double box, double inv_box) {
    if (BOX) return fma(-box, rint(d * inv_box), d);
    return d;
}

// |d|^2 in FP32 with exact products (FMA) and compensated summation; the
// displacement itself is formed in FP64 and rounded to FP32 once.
__device__ __forceinline__ double sqlen_f32c(double dx, double dy, double dz) {
#pragma clang fp contract(off)
    const float x = (float)dx, y = (float)dy, z = (float)dz;
    const float px = x * x, ex = fmaf(x, x, -px);
    const float py = y * y, ey = fmaf(y, y, -py);
    const float pz = z * z, ez = fmaf(z, z, -pz);
    float s1 = px + py;
    float bb = s1 - px;
    const float e1 = (px - (s1 - bb)) + (py - bb);
    const float s2 = s1 + pz;
    bb = s2 - s1;
    const float e2 = (s1 - (s2 - bb)) + (pz - bb);
    const float lo = ((ex + ey) + ez) + (e1 + e2);
    return (double)s2 + (double)lo;
}

template <bool MIXED>
__device__ __forceinline__ double sqlen(double dx, double dy, double dz) {
    if (MIXED) return sqlen_f32c(dx, dy, dz);
    return fma(dx, dx, fma(dy, dy, dz * dz));
}

__device__ __forceinline__ double block_sum(double v, double *red) {
    const int t = threadIdx.x, T = blockDim.x; // T is a power of two
    red[t] = v;
    __syncthreads();
    for (int s = T >> 1; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ void set_flag(int32_t *flags, int bits) {
    __hip_atomic_fetch_or(flags, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// LDS map (doubles): [0,CH) x | [CH,2CH) y | [2CH,3CH) z | [3CH,4CH) lambda |
// [4CH, 4CH+T) reduction | then 2 broadcast mantissas, 2 broadcast exponents.
__device__ __forceinline__ double *zslot_m(double *sm) { return sm + 4 * CH + blockDim.x; }
__device__ __forceinline__ int *zslot_e(double *sm) { return (int *)(sm + 4 * CH + blockDim.x + 2); }

// Extended-exponent accumulate: (A, e) += tm * 2^te, rescaling the running
// sum to the larger exponent; W (term-weighted displacements) shares the
// scale of A.
// w = w * f + d, written in place.  Plain C++ lets the compiler pick the
// two-address v_fmac form with d as the accumulator, which costs a register
// copy per update for the loop-carried w; the explicit three-address form
// avoids it.  Pure arithmetic, no memory access.
__device__ __forceinline__ void fma_inplace(double &w, double f, double d) {
    asm("v_fma_f64 %0, %0, %1, %2" : "+v"(w) : "v"(f), "v"(d));
}

// Opaque copy: keeps the compiler from merging the owner's displacement with
// the identical expression in the per-row update, which it would otherwise
// hoist above both branches and evaluate for finished rows too.
__device__ __forceinline__ double opaque(double x) {
    asm("" : "+v"(x));
    return x;
}

template <bool WSUM>
__device__ __forceinline__ void xacc(double &A, int &e, double &Wx, double &Wy, double &Wz, double tm, int te,
                                     double dx, double dy, double dz) {
    const int en = max(e, te);
    const double fo = ldexp(1.0, e - en);
    const double tn = ldexp(tm, te - en);
    fma_inplace(A, fo, tn);
    if (WSUM) {
        fma_inplace(Wx, fo, tn * dx);
        fma_inplace(Wy, fo, tn * dy);
        fma_inplace(Wz, fo, tn * dz);
    }
    e = en;
}

// 2^x as mantissa p in [0.7, 1.42] and integer exponent n, x >= XLO.
__device__ __forceinline__ void exp2x(double x, double &p, int &n) {
    x = fmax(x, XLO);
    const double r = rint(x);
    p = exp2_frac(x - r);
    n = (int)r;
}

// --------------------------------------------------------------- forward
// Accumulator v (0-based q) sums Z_f[u-1] K(u, v) over u <= v, u = s + 1 at
// step s, with K(u,v) = 2^(kappa |r_v^P - r_u^1|^2 + h_v) and
// h_v = -kappa |r_v^P - r_ref^1|^2, ref = v+1 (v < N) or v (v = N).
// The diagonal K(v,v) does not depend on the recursion and is precomputed,
// so the owner of step s only multiplies, adds, rescales and broadcasts
// before the other terms of the step are formed.  Owners keep their results
// in registers; nothing is written to global memory inside the step loop.
template <int J, bool BOX, bool MIXED, bool WSUM>
__device__ void forward_role(const LaunchArgs &a, const SysDesc sd, double *sm) {
    // J <= 4: owners keep results in registers until the loop ends; J = 8
    // has no registers to spare and stores them as they are produced.
    constexpr bool DEFER = J <= 4;
    const int t = threadIdx.x, T = blockDim.x, N = sd.N;
    const size_t NN = (size_t)N;
    const double *__restrict__ b1 = a.pos + sd.off;                        // bead 1 plane
    const double *__restrict__ bP = a.pos + sd.off + (size_t)(sd.P - 1) * 3 * NN; // bead P plane
    double *sx = sm, *sy = sm + CH, *sz = sm + 2 * CH;
    double *zsm = zslot_m(sm);
    int *zse = zslot_e(sm);
    const double kap = sd.kappa, box = a.box, ib = a.inv_box;

    double *base = (a.mode & M_SAVE) ? a.state + sd.st : a.ws + sd.ws;
    double *__restrict__ zm_out = base + ((a.mode & M_SAVE) ? StLayout::zf_m(N) : WsLayout::zf_m(N));
    double *__restrict__ ze_out = base + ((a.mode & M_SAVE) ? StLayout::zf_e(N) : WsLayout::zf_e(N));
    double *__restrict__ r_out = base + ((a.mode & M_SAVE) ? StLayout::rf(N) : WsLayout::rf(N));

    double px[J], py[J], pz[J], hl[J], pd[J], iv[DEFER ? J : 1], A[J], Wx[J], Wy[J], Wz[J], om[DEFER ? J : 1];
    int e[J], kd[J], oe[DEFER ? J : 1];
    bool range_bad = false;
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int q = t + j * T;
        px[j] = py[j] = pz[j] = hl[j] = pd[j] = 0.0;
        kd[j] = 0;
        if (DEFER) {
            om[j] = 0.0;
            oe[j] = 0;
            iv[j] = 1.0 / (double)(q + 1);
        }
        if (q < N) {
            px[j] = bP[q];
            py[j] = bP[NN + q];
            pz[j] = bP[2 * NN + q];
            const int r = q < N - 1 ? q + 1 : q;
            const double ql = sqlen<MIXED>(mimg<BOX>(px[j] - b1[r], box, ib), mimg<BOX>(py[j] - b1[NN + r], box, ib),
                                           mimg<BOX>(pz[j] - b1[2 * NN + r], box, ib));
            hl[j] = -kap * ql;
            range_bad |= !(hl[j] <= XHI);
            const double qs = sqlen<MIXED>(mimg<BOX>(px[j] - b1[q], box, ib), mimg<BOX>(py[j] - b1[NN + q], box, ib),
                                           mimg<BOX>(pz[j] - b1[2 * NN + q], box, ib));
            exp2x(fma(kap, qs, hl[j]), pd[j], kd[j]);
        }
        A[j] = 0.0;
        Wx[j] = Wy[j] = Wz[j] = 0.0;
        e[j] = EMIN;
    }
    if (range_bad) set_flag(a.flags, ST_RANGE);
    if (t == 0) {
        zsm[0] = 1.0; // Z_f[0] = 1  (V^[1,0] = 0)
        zse[0] = 0;
    }
    int jo = 0, to = 0; // owner of step s: row jo, thread to (s = jo*T + to)
    for (int s = 0; s < N; ++s) {
        const int li = s % CH;
        if (li == 0) {
            const int n = min(CH, N - s);
            for (int i = t; i < n; i += T) {
                sx[i] = b1[s + i];
                sy[i] = b1[NN + s + i];
                sz[i] = b1[2 * NN + s + i];
            }
            __syncthreads();
        }
        const int slot = s & 1;
        const double zm = zsm[slot];
        const int ze = zse[slot];
        const double ux = sx[li], uy = sy[li], uz = sz[li];
        const bool own = t == to;
        // owner of step s: diagonal term, Z_f[s+1] = A / (s+1), broadcast
#pragma unroll
        for (int j = 0; j < J; ++j) {
            if (j == jo && own) {
                const double dx = mimg<BOX>(px[j] - opaque(ux), box, ib);
                const double dy = mimg<BOX>(py[j] - opaque(uy), box, ib);
                const double dz = mimg<BOX>(pz[j] - opaque(uz), box, ib);
                xacc<WSUM>(A[j], e[j], Wx[j], Wy[j], Wz[j], zm * pd[j], ze + kd[j], dx, dy, dz);
                const double zz = DEFER ? A[j] * iv[DEFER ? j : 0] : A[j] / (double)(s + 1);
                const double mz = __builtin_amdgcn_frexp_mant(zz);
                const int zx = e[j] + __builtin_amdgcn_frexp_exp(zz);
                zsm[slot ^ 1] = mz;
                zse[slot ^ 1] = zx;
                if (DEFER) {
                    om[DEFER ? j : 0] = mz;
                    oe[DEFER ? j : 0] = zx;
                } else {
                    zm_out[s + 1] = mz;
                    ze_out[s + 1] = (double)zx;
                    if (WSUM) {
                        const double ia = 1.0 / A[j];
                        r_out[s] = Wx[j] * ia;
                        r_out[NN + s] = Wy[j] * ia;
                        r_out[2 * NN + s] = Wz[j] * ia;
                    }
                }
            }
        }
        // every later accumulator v > s adds Z_f[s] K(s+1, v)
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int q = t + j * T;
            if (q > s && q < N) {
                const double dx = mimg<BOX>(px[j] - ux, box, ib);
                const double dy = mimg<BOX>(py[j] - uy, box, ib);
                const double dz = mimg<BOX>(pz[j] - uz, box, ib);
                double p;
                int kx;
                exp2x(fma(kap, sqlen<MIXED>(dx, dy, dz), hl[j]), p, kx);
                xacc<WSUM>(A[j], e[j], Wx[j], Wy[j], Wz[j], zm * p, ze + kx, dx, dy, dz);
            }
        }
        if (++to == T) {
            to = 0;
            ++jo;
        }
        __syncthreads();
    }
    // results: Z_f[v] (v = 1..N) and the forward-weighted mean displacement
    if (t == 0) {
        zm_out[0] = 1.0;
        ze_out[0] = 0.0;
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int q = t + j * T;
        if (DEFER && q < N) {
            zm_out[q + 1] = om[DEFER ? j : 0];
            ze_out[q + 1] = (double)oe[DEFER ? j : 0];
            if (WSUM) {
                const double ia = 1.0 / A[j];
                r_out[q] = Wx[j] * ia;
                r_out[NN + q] = Wy[j] * ia;
                r_out[2 * NN + q] = Wz[j] * ia;
            }
        }
    }
}

// --------------------------------------------------------------- backward
// Accumulator u (0-based q) sums (Z_b[l+1]/l) K(u, l) over l >= u, l = s + 1
// at step s (descending), K(u,l) = 2^(kappa |r_l^P - r_u^1|^2 + h_l); h_l is
// staged in LDS with the bead-P positions.  Diagonal precomputed as in the
// forward recursion.
template <int J, bool BOX, bool MIXED>
__device__ void backward_role(const LaunchArgs &a, const SysDesc sd, double *sm) {
    constexpr bool DEFER = J <= 4;
    const int t = threadIdx.x, T = blockDim.x, N = sd.N;
    const size_t NN = (size_t)N;
    const double *__restrict__ b1 = a.pos + sd.off;
    const double *__restrict__ bP = a.pos + sd.off + (size_t)(sd.P - 1) * 3 * NN;
    double *sx = sm, *sy = sm + CH, *sz = sm + 2 * CH, *sh = sm + 3 * CH;
    double *zsm = zslot_m(sm);
    int *zse = zslot_e(sm);
    const double kap = sd.kappa, box = a.box, ib = a.inv_box;

    double *base = a.ws + sd.ws;
    double *__restrict__ zm_out = base + WsLayout::zb_m(N);
    double *__restrict__ ze_out = base + WsLayout::zb_e(N);
    double *__restrict__ r_out = base + WsLayout::rb(N);

    double px[J], py[J], pz[J], pd[J], iv[DEFER ? J : 1], A[J], Wx[J], Wy[J], Wz[J];
    int e[J], kd[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int q = t + j * T;
        px[j] = py[j] = pz[j] = pd[j] = 0.0;
        kd[j] = 0;
        if (DEFER) iv[j] = q > 0 ? 1.0 / (double)q : 0.0;
        if (q < N) {
            px[j] = b1[q];
            py[j] = b1[NN + q];
            pz[j] = b1[2 * NN + q];
            const double vx = bP[q], vy = bP[NN + q], vz = bP[2 * NN + q];
            const int r = q < N - 1 ? q + 1 : q;
            const double ql = sqlen<MIXED>(mimg<BOX>(vx - b1[r], box, ib), mimg<BOX>(vy - b1[NN + r], box, ib),
                                           mimg<BOX>(vz - b1[2 * NN + r], box, ib));
            const double qs = sqlen<MIXED>(mimg<BOX>(vx - px[j], box, ib), mimg<BOX>(vy - py[j], box, ib),
                                           mimg<BOX>(vz - pz[j], box, ib));
            exp2x(fma(kap, qs, -kap * ql), pd[j], kd[j]);
        }
        A[j] = 0.0;
        Wx[j] = Wy[j] = Wz[j] = 0.0;
        e[j] = EMIN;
    }
    if (t == 0) {
        const double zz = 1.0 / (double)N; // broadcast Z_b[N+1] / N, Z_b[N+1] = 1
        zsm[(N - 1) & 1] = __builtin_amdgcn_frexp_mant(zz);
        zse[(N - 1) & 1] = __builtin_amdgcn_frexp_exp(zz);
    }
    bool range_bad = false;
    int jo = (N - 1) / T, to = (N - 1) - jo * T; // owner of step s
    for (int s = N - 1; s >= 0; --s) {
        const int lo = s - s % CH;
        if (s == N - 1 || s % CH == CH - 1) {
            const int n = s - lo + 1;
            for (int i = t; i < n; i += T) {
                const int l = lo + i;
                const double x = bP[l], y = bP[NN + l], z = bP[2 * NN + l];
                const int r = l < N - 1 ? l + 1 : l;
                const double dx = mimg<BOX>(x - b1[r], box, ib);
                const double dy = mimg<BOX>(y - b1[NN + r], box, ib);
                const double dz = mimg<BOX>(z - b1[2 * NN + r], box, ib);
                const double h = -kap * sqlen<MIXED>(dx, dy, dz);
                range_bad |= !(h <= XHI);
                sx[i] = x;
                sy[i] = y;
                sz[i] = z;
                sh[i] = h;
            }
            __syncthreads();
        }
        const bool own = t == to;
        const int li = s - lo;
        const int slot = s & 1;
        const double zm = zsm[slot];
        const int ze = zse[slot];
        const double ux = sx[li], uy = sy[li], uz = sz[li], h = sh[li];
        // owner of step s: Z_b[s+1] = A; broadcast Z_b[s+1] / s
#pragma unroll
        for (int j = 0; j < J; ++j) {
            if (j == jo && own) {
                const double dx = mimg<BOX>(opaque(ux) - px[j], box, ib);
                const double dy = mimg<BOX>(opaque(uy) - py[j], box, ib);
                const double dz = mimg<BOX>(opaque(uz) - pz[j], box, ib);
                xacc<true>(A[j], e[j], Wx[j], Wy[j], Wz[j], zm * pd[j], ze + kd[j], dx, dy, dz);
                const double zz = DEFER ? A[j] * iv[DEFER ? j : 0] : (s > 0 ? A[j] / (double)s : 0.0);
                zsm[slot ^ 1] = __builtin_amdgcn_frexp_mant(zz);
                zse[slot ^ 1] = e[j] + __builtin_amdgcn_frexp_exp(zz);
                if (!DEFER) {
                    zm_out[s + 1] = __builtin_amdgcn_frexp_mant(A[j]);
                    ze_out[s + 1] = (double)(e[j] + __builtin_amdgcn_frexp_exp(A[j]));
                    const double ia = 1.0 / A[j];
                    r_out[s] = Wx[j] * ia;
                    r_out[NN + s] = Wy[j] * ia;
                    r_out[2 * NN + s] = Wz[j] * ia;
                }
            }
        }
        // every earlier accumulator u < s adds (Z_b[s+2]/(s+1)) K(u, s+1)
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int q = t + j * T;
            if (q < s) {
                const double dx = mimg<BOX>(ux - px[j], box, ib);
                const double dy = mimg<BOX>(uy - py[j], box, ib);
                const double dz = mimg<BOX>(uz - pz[j], box, ib);
                double p;
                int kx;
                exp2x(fma(kap, sqlen<MIXED>(dx, dy, dz), h), p, kx);
                xacc<true>(A[j], e[j], Wx[j], Wy[j], Wz[j], zm * p, ze + kx, dx, dy, dz);
            }
        }
        if (--to < 0) {
            to = T - 1;
            --jo;
        }
        __syncthreads();
    }
    if (range_bad) set_flag(a.flags, ST_RANGE);
    // results: Z_b[u] (u = 1..N+1) and the backward-weighted mean displacement
    if (t == 0) {
        zm_out[N + 1] = 1.0;
        ze_out[N + 1] = 0.0;
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int q = t + j * T;
        if (DEFER && q < N) {
            zm_out[q + 1] = __builtin_amdgcn_frexp_mant(A[j]);
            ze_out[q + 1] = (double)(e[j] + __builtin_amdgcn_frexp_exp(A[j]));
            const double ia = 1.0 / A[j];
            r_out[q] = Wx[j] * ia;
            r_out[NN + q] = Wy[j] * ia;
            r_out[2 * NN + q] = Wz[j] * ia;
        }
    }
}

// ---------------------------------------------------------------- springs
// One thread per particle, loop over beads.  Interior energies E_int(l)
// (Theory, "Reducing the potential", interior springs j = 1..P-1), interior
// bead forces -m w_P^2 (2 r^j - r^{j+1} - r^{j-1}) for j = 2..P-1 (Theory,
// "Force on interior beads"), and the optional trap.  In distinguishable mode
// every ring closes on itself and all beads are written here.
template <bool BOX>
__device__ void springs_role(const LaunchArgs &a, const SysDesc sd, int si, int chunk, double *sm) {
    const int t = threadIdx.x, T = blockDim.x, N = sd.N, P = sd.P;
    const size_t NN = (size_t)N;
    const int q = chunk * T + t;
    const bool dist = (a.mode & M_DIST) != 0;
    const bool wf = (a.mode & M_FORCES) && a.out;
    const double box = a.box, ib = a.inv_box;
    const double k = sd.k, mw2 = sd.mw2;
    const double trapc = sd.m * a.trap_w2 / (double)P; // force coefficient
    const double scale = (a.mode & M_ADJOINT) ? -a.gscale[si] : 1.0;
    double esum = 0.0;
    bool bad = false;
    if (q < N) {
        const double *p0 = a.pos + sd.off;
        double *fo = wf ? a.out + sd.off : nullptr;
        double cx = p0[q], cy = p0[NN + q], cz = p0[2 * NN + q];
        double vx, vy, vz; // previous bead
        if (dist) {
            const size_t o = (size_t)(P - 1) * 3 * NN;
            vx = p0[o + q];
            vy = p0[o + NN + q];
            vz = p0[o + 2 * NN + q];
        } else {
            vx = cx; vy = cy; vz = cz;
        }
        double ei = 0.0, et = 0.0;
        for (int j = 0; j < P; ++j) {
            bad |= !isfinite(cx) || !isfinite(cy) || !isfinite(cz);
            double nx, ny, nz;
            if (j + 1 < P) {
                const size_t o = (size_t)(j + 1) * 3 * NN;
                nx = p0[o + q];
                ny = p0[o + NN + q];
                nz = p0[o + 2 * NN + q];
            } else {
                nx = p0[q];
                ny = p0[NN + q];
                nz = p0[2 * NN + q];
            }
            const double ax = mimg<BOX>(cx - nx, box, ib);
            const double ay = mimg<BOX>(cy - ny, box, ib);
            const double az = mimg<BOX>(cz - nz, box, ib);
            if (j + 1 < P || dist) ei += ax * ax + ay * ay + az * az;
            et += cx * cx + cy * cy + cz * cz;
            if (wf && ((j > 0 && j < P - 1) || dist)) {
                const double bx = mimg<BOX>(cx - vx, box, ib);
                const double by = mimg<BOX>(cy - vy, box, ib);
                const double bz = mimg<BOX>(cz - vz, box, ib);
                const size_t o = (size_t)j * 3 * NN;
                fo[o + q] = scale * (-mw2 * (ax + bx) - trapc * cx);
                fo[o + NN + q] = scale * (-mw2 * (ay + by) - trapc * cy);
                fo[o + 2 * NN + q] = scale * (-mw2 * (az + bz) - trapc * cz);
            }
            vx = cx; vy = cy; vz = cz;
            cx = nx; cy = ny; cz = nz;
        }
        esum = k * ei + 0.5 * trapc * et;
    }
    if (bad) set_flag(a.flags, ST_NONFINITE_IN);
    const double tot = block_sum(esum, sm + 4 * CH);
    if (t == 0) a.ws[sd.ws + WsLayout::epart(N) + chunk] = tot;
}

// ---------------------------------------------------------------- finalize
// Run by the last workgroup of a system to arrive.  Exterior-bead forces
// (Theory, "Force on exterior beads") written in displacement form:
//   F_l^P = -m w^2 [ (r_l^P - r_l^{P-1}) + sum_{u<=l} Pr[l->u] (r_l^P - r_u^1)
//                    + Pr[l->l+1] (r_l^P - r_{l+1}^1) ]
//   F_l^1 = -m w^2 [ (r_l^1 - r_l^2) - sum_{l'>=l} Pr[l'->l] (r_l'^P - r_l^1)
//                    - Pr[l-1->l] (r_{l-1}^P - r_l^1) ]
// using that each row and each column of Pr sums to one.  The two Pr sums
// are rho * (weighted mean displacement) from the recursions.  Energy:
//   V^[1,N] = sum_l E_int(l) + sum_{l<N} s(l,l+1) + s(N,N) - ln(Z_f[N]) / beta.
template <bool BOX>
__device__ void finalize(const LaunchArgs &a, const SysDesc sd, int si, double *sm) {
    const int t = threadIdx.x, T = blockDim.x, N = sd.N, P = sd.P;
    const size_t NN = (size_t)N;
    const double *p0 = a.pos + sd.off;
    const double box = a.box, ib = a.inv_box;
    const bool dist = (a.mode & M_DIST) != 0;
    const bool wf = (a.mode & M_FORCES) && a.out && !dist;
    const bool we = (a.mode & M_ENERGY) && a.energy;
    const double *wsb = a.ws + sd.ws;
    const double *fsrc = (a.mode & M_ADJOINT) ? a.state + sd.st : a.ws + sd.ws;
    const double *zfm = fsrc + ((a.mode & M_ADJOINT) ? StLayout::zf_m(N) : WsLayout::zf_m(N));
    const double *zfe = fsrc + ((a.mode & M_ADJOINT) ? StLayout::zf_e(N) : WsLayout::zf_e(N));
    const double *rf = fsrc + ((a.mode & M_ADJOINT) ? StLayout::rf(N) : WsLayout::rf(N));
    const double *zbm = wsb + WsLayout::zb_m(N);
    const double *zbe = wsb + WsLayout::zb_e(N);
    const double *rb = wsb + WsLayout::rb(N);
    const double scale = (a.mode & M_ADJOINT) ? -a.gscale[si] : 1.0;
    const double mw2 = sd.mw2;
    const double trapc = sd.m * a.trap_w2 / (double)P;
    const size_t oP = (size_t)(P - 1) * 3 * NN, oQ = (size_t)(P - 2) * 3 * NN, o2 = 3 * NN;
    double elink = 0.0;
    bool bad = false;
    if (!dist) {
        const double nInv = 1.0 / zfm[N];
        const int ne = (int)zfe[N];
        for (int q = t; q < N; q += T) {
            const double Px = p0[oP + q], Py = p0[oP + NN + q], Pz = p0[oP + 2 * NN + q];
            const double Fx = p0[q], Fy = p0[NN + q], Fz = p0[2 * NN + q];
            // link (or closing) spring of q: bead P of q to bead 1 of q+1 (q itself if last)
            const int r = q < N - 1 ? q + 1 : q;
            const double lx = mimg<BOX>(Px - p0[r], box, ib);
            const double ly = mimg<BOX>(Py - p0[NN + r], box, ib);
            const double lz = mimg<BOX>(Pz - p0[2 * NN + r], box, ib);
            elink += lx * lx + ly * ly + lz * lz;
            if (!wf) continue;
            // rho_l = Z_f[l] Z_b[l+1] / Z_f[N] for l = q+1 and l = q
            double rho, plink;
            if (q == N - 1) {
                rho = 1.0;
                plink = 0.0;
            } else {
                rho = ldexp(zfm[q + 1] * zbm[q + 2] * nInv, (int)zfe[q + 1] + (int)zbe[q + 2] - ne);
                plink = 1.0 - rho;
            }
            const double rhop = ldexp(zfm[q] * zbm[q + 1] * nInv, (int)zfe[q] + (int)zbe[q + 1] - ne);
            const double plinkp = q > 0 ? 1.0 - rhop : 0.0;
            // bead P
            const double ix = mimg<BOX>(Px - p0[oQ + q], box, ib);
            const double iy = mimg<BOX>(Py - p0[oQ + NN + q], box, ib);
            const double iz = mimg<BOX>(Pz - p0[oQ + 2 * NN + q], box, ib);
            double gx = ix + rho * rf[q] + plink * lx;
            double gy = iy + rho * rf[NN + q] + plink * ly;
            double gz = iz + rho * rf[2 * NN + q] + plink * lz;
            const double fPx = scale * (-mw2 * gx - trapc * Px);
            const double fPy = scale * (-mw2 * gy - trapc * Py);
            const double fPz = scale * (-mw2 * gz - trapc * Pz);
            // bead 1
            const double jx = mimg<BOX>(Fx - p0[o2 + q], box, ib);
            const double jy = mimg<BOX>(Fy - p0[o2 + NN + q], box, ib);
            const double jz = mimg<BOX>(Fz - p0[o2 + 2 * NN + q], box, ib);
            double hx = jx - rhop * rb[q], hy = jy - rhop * rb[NN + q], hz = jz - rhop * rb[2 * NN + q];
            if (q > 0) {
                const double kx = mimg<BOX>(p0[oP + q - 1] - Fx, box, ib);
                const double ky = mimg<BOX>(p0[oP + NN + q - 1] - Fy, box, ib);
                const double kz = mimg<BOX>(p0[oP + 2 * NN + q - 1] - Fz, box, ib);
                hx -= plinkp * kx;
                hy -= plinkp * ky;
                hz -= plinkp * kz;
            }
            const double f1x = scale * (-mw2 * hx - trapc * Fx);
            const double f1y = scale * (-mw2 * hy - trapc * Fy);
            const double f1z = scale * (-mw2 * hz - trapc * Fz);
            bad |= !isfinite(fPx) || !isfinite(fPy) || !isfinite(fPz) || !isfinite(f1x) ||
                   !isfinite(f1y) || !isfinite(f1z);
            double *o = a.out + sd.off;
            o[q] = f1x;
            o[NN + q] = f1y;
            o[2 * NN + q] = f1z;
            o[oP + q] = fPx;
            o[oP + NN + q] = fPy;
            o[oP + 2 * NN + q] = fPz;
        }
    }
    if (we) {
        const double links = block_sum(elink, sm + 4 * CH);
        if (t == 0) {
            double E = 0.0;
            for (int c = 0; c < sd.nchunk; ++c) E += wsb[WsLayout::epart(N) + c];
            if (!dist) E += sd.k * links - (log(zfm[N]) + zfe[N] * LN2) / sd.beta;
            bad |= !isfinite(E);
            a.energy[si] = E;
        }
    }
    if (bad) set_flag(a.flags, ST_NONFINITE_OUT);
}

// ------------------------------------------------------------ fused kernel
template <int J, bool BOX, bool MIXED>
__device__ __forceinline__ void exchange_body(const LaunchArgs &a) {
    extern __shared__ double sm[];
    __shared__ int s_last;
    const Item it = a.items[blockIdx.x];
    const SysDesc sd = a.sys[it.sys];
    if (it.role == ROLE_FORWARD) {
        if (a.mode & M_WSUM)
            forward_role<J, BOX, MIXED, true>(a, sd, sm);
        else
            forward_role<J, BOX, MIXED, false>(a, sd, sm);
    } else if (it.role == ROLE_BACKWARD) {
        backward_role<J, BOX, MIXED>(a, sd, sm);
    } else {
        springs_role<BOX>(a, sd, it.sys, it.idx, sm);
    }
    // Arrival: release this workgroup's global writes, count it, and let the
    // last workgroup of the system (acquire) compute the exterior forces.
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const int target = ((a.mode & M_FWD) ? 1 : 0) + ((a.mode & M_BWD) ? 1 : 0) + sd.nchunk;
        const int old = __hip_atomic_fetch_add(&a.counters[it.sys], 1, __ATOMIC_ACQ_REL,
                                               __HIP_MEMORY_SCOPE_AGENT);
        s_last = (old == target - 1);
    }
    __syncthreads();
    if (s_last) {
        __threadfence();
        finalize<BOX>(a, sd, it.sys, sm);
        if (threadIdx.x == 0)
            __hip_atomic_store(&a.counters[it.sys], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Register budget: J <= 2 keeps 4 waves per SIMD at 1024 threads; J = 4 and
// J = 8 need the 512-thread bound to avoid spilling.
template <int J, bool BOX, bool MIXED>
__global__ void __launch_bounds__(1024) k_exchange(LaunchArgs a) {
    exchange_body<J, BOX, MIXED>(a);
}

template <int J, bool BOX, bool MIXED>
__global__ void __launch_bounds__(512) k_exchange_wide(LaunchArgs a) {
    exchange_body<J, BOX, MIXED>(a);
}

size_t exchange_smem_bytes(int threads) { return (size_t)(4 * CH + threads + 4) * sizeof(double); }

template <bool BOX, bool MIXED>
static hipError_t launch_j(const LaunchArgs &a, int nitems, int threads, int per_thread, hipStream_t st) {
    const size_t smem = exchange_smem_bytes(threads);
    switch (per_thread) {
    case 1:
        hipLaunchKernelGGL((k_exchange<1, BOX, MIXED>), dim3(nitems), dim3(threads), smem, st, a);
        break;
    case 2:
        hipLaunchKernelGGL((k_exchange<2, BOX, MIXED>), dim3(nitems), dim3(threads), smem, st, a);
        break;
    case 4:
        if (threads > 512) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_exchange_wide<4, BOX, MIXED>), dim3(nitems), dim3(threads), smem, st, a);
        break;
    case 8:
        if (threads > 512) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_exchange_wide<8, BOX, MIXED>), dim3(nitems), dim3(threads), smem, st, a);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_exchange(const LaunchArgs &a, int nitems, int threads, int per_thread, hipStream_t st) {
    if (nitems <= 0) return hipSuccess;
    const bool box = a.box > 0;
    if (box) return a.mixed ? launch_j<true, true>(a, nitems, threads, per_thread, st)
                            : launch_j<true, false>(a, nitems, threads, per_thread, st);
    return a.mixed ? launch_j<false, true>(a, nitems, threads, per_thread, st)
                   : launch_j<false, false>(a, nitems, threads, per_thread, st);
}

// ----------------------------------------------------------- small kernels
__global__ void k_clear(int32_t *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

hipError_t launch_clear(int32_t *p, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + 255) / 256;
    const int blocks = (int)(nb < 1024 ? nb : 1024);
    hipLaunchKernelGGL(k_clear, dim3(blocks), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

// Velocity-Verlet half kick (and drift): v += dt/(2m) f; x += dt v.
__global__ void k_md_update(const SysDesc *sys, const EChunk *ch, double *pos, double *vel, const double *f,
                            double dt, int drift) {
    const EChunk c = ch[blockIdx.x];
    const double h = 0.5 * dt / sys[c.sys].m;
    for (int64_t i = c.begin + threadIdx.x; i < c.end; i += blockDim.x) {
        const double v = fma(h, f[i], vel[i]);
        vel[i] = v;
        if (drift) pos[i] = fma(dt, v, pos[i]);
    }
}

hipError_t launch_md_update(const SysDesc *sys, const EChunk *chunks, int nchunks, double *pos, double *vel,
                            const double *forces, double dt, int drift, hipStream_t st) {
    if (nchunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_md_update, dim3(nchunks), dim3(256), 0, st, sys, chunks, pos, vel, forces, dt, drift);
    return hipGetLastError();
}

// ------------------------------------------------------------ debug exports
// Gauge constants c_l = E_int(l) + lambda_l and their prefix sums
// cpre[v] = sum_{l<=v} c_l (1-based), serial scan by one thread.
template <bool BOX>
__global__ void k_debug_prefix(LaunchArgs a, int si) {
    const SysDesc &sd = a.sys[si];
    const int N = sd.N, P = sd.P, t = threadIdx.x, T = blockDim.x;
    const size_t NN = (size_t)N;
    const double *p0 = a.pos + sd.off;
    double *cpre = a.ws + sd.ws + WsLayout::cpre(N, sd.nchunk);
    const double box = a.box, ib = a.inv_box;
    for (int q = t; q < N; q += T) {
        double ei = 0.0;
        for (int j = 0; j + 1 < P; ++j) {
            const size_t o = (size_t)j * 3 * NN, o1 = (size_t)(j + 1) * 3 * NN;
            const double dx = mimg<BOX>(p0[o1 + q] - p0[o + q], box, ib);
            const double dy = mimg<BOX>(p0[o1 + NN + q] - p0[o + NN + q], box, ib);
            const double dz = mimg<BOX>(p0[o1 + 2 * NN + q] - p0[o + 2 * NN + q], box, ib);
            ei += dx * dx + dy * dy + dz * dz;
        }
        const size_t oP = (size_t)(P - 1) * 3 * NN;
        const int r = q < N - 1 ? q + 1 : q;
        const double dx = mimg<BOX>(p0[oP + q] - p0[r], box, ib);
        const double dy = mimg<BOX>(p0[oP + NN + q] - p0[NN + r], box, ib);
        const double dz = mimg<BOX>(p0[oP + 2 * NN + q] - p0[2 * NN + r], box, ib);
        cpre[q + 1] = sd.k * (ei + dx * dx + dy * dy + dz * dz);
    }
    __syncthreads();
    if (t == 0) {
        cpre[0] = 0.0;
        for (int v = 1; v <= N; ++v) cpre[v] += cpre[v - 1];
    }
}

hipError_t launch_debug_prefix(const LaunchArgs &a, int s, int threads, hipStream_t st) {
    if (a.box > 0)
        hipLaunchKernelGGL(k_debug_prefix<true>, dim3(1), dim3(threads), 0, st, a, s);
    else
        hipLaunchKernelGGL(k_debug_prefix<false>, dim3(1), dim3(threads), 0, st, a, s);
    return hipGetLastError();
}

// One thread per table entry (debug only).
template <bool BOX>
__global__ void k_debug_table(LaunchArgs a, int si, int what, double *dst) {
    const SysDesc &sd = a.sys[si];
    const int N = sd.N;
    const size_t NN = (size_t)N;
    const double *p0 = a.pos + sd.off;
    const double *bP = p0 + (size_t)(sd.P - 1) * 3 * NN;
    const double *ws = a.ws + sd.ws;
    const double *cpre = ws + WsLayout::cpre(N, sd.nchunk);
    const double *zfm = ws + WsLayout::zf_m(N), *zfe = ws + WsLayout::zf_e(N);
    const double *zbm = ws + WsLayout::zb_m(N), *zbe = ws + WsLayout::zb_e(N);
    const double box = a.box, ib = a.inv_box;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (what == 3) { // V^[1,v], v = 0..N
        if (idx > N) return;
        dst[idx] = cpre[idx] - (log(zfm[idx]) + zfe[idx] * LN2) / sd.beta;
        return;
    }
    if (what == 4) { // V^[u,N], u = 1..N+1; index 0 is 0
        if (idx > N + 1) return;
        dst[idx] = idx == 0 ? 0.0 : (cpre[N] - cpre[idx - 1]) - (log(zbm[idx]) + zbe[idx] * LN2) / sd.beta;
        return;
    }
    if (idx >= (int64_t)N * N) return;
    const int row = (int)(idx / N), col = (int)(idx % N); // 0-based
    // spring exponent pieces for (v = row or col as needed)
    auto q2 = [&](int v, int u) { // |r_v^P - r_u^1|^2 (0-based)
        const double dx = mimg<BOX>(bP[v] - p0[u], box, ib);
        const double dy = mimg<BOX>(bP[NN + v] - p0[NN + u], box, ib);
        const double dz = mimg<BOX>(bP[2 * NN + v] - p0[2 * NN + u], box, ib);
        return dx * dx + dy * dy + dz * dz;
    };
    if (what == 2) { // E^[u,v] at [u-1][v-1], u = row+1, v = col+1
        if (row > col) {
            dst[idx] = 0.0;
            return;
        }
        const int v = col, u = row;
        const int r = v < N - 1 ? v + 1 : v;
        dst[idx] = (cpre[v + 1] - cpre[u]) + sd.k * (q2(v, u) - q2(v, r));
        return;
    }
    // what == 1: Pr[l -> l'] at [l-1][l'-1], l = row+1, l' = col+1
    const int l = row, u = col;
    const double nInv = 1.0 / zfm[N];
    const int ne = (int)zfe[N];
    if (u == l + 1) {
        const double rho = ldexp(zfm[l + 1] * zbm[l + 2] * nInv, (int)zfe[l + 1] + (int)zbe[l + 2] - ne);
        dst[idx] = 1.0 - rho;
    } else if (u <= l) {
        const int r = l < N - 1 ? l + 1 : l;
        double p;
        int nr;
        exp2x(fma(sd.kappa, q2(l, u), -sd.kappa * q2(l, r)), p, nr);
        dst[idx] = ldexp(zfm[u] * p * zbm[l + 2] * nInv / (double)(l + 1),
                         (int)zfe[u] + nr + (int)zbe[l + 2] - ne);
    } else {
        dst[idx] = 0.0;
    }
}

hipError_t launch_debug_table(const LaunchArgs &a, int s, int N, int what, double *dst, hipStream_t st) {
    const int64_t n = (what == 3 || what == 4) ? (int64_t)N + 2 : (int64_t)N * N;
    const int blocks = (int)((n + 255) / 256);
    if (a.box > 0)
        hipLaunchKernelGGL(k_debug_table<true>, dim3(blocks), dim3(256), 0, st, a, s, what, dst);
    else
        hipLaunchKernelGGL(k_debug_table<false>, dim3(blocks), dim3(256), 0, st, a, s, what, dst);
    return hipGetLastError();
}

// ------------------------------------------------- endpoint spring table
// s(v,u) = k |r_v^P - r_u^1|^2 for u <= v, packed lower triangle by rows.
// 64 x 64 tiles of the triangle, endpoint tiles staged in LDS; each thread
// writes consecutive u of one row (coalesced row segments).
template <bool BOX, bool F32>
__global__ void __launch_bounds__(256) k_endpoint_springs(LaunchArgs a, int si, void *dst) {
    constexpr int TB = 64;
    __shared__ double rv[3][TB], ru[3][TB];
    const SysDesc &sd = a.sys[si];
    const int N = sd.N;
    const size_t NN = (size_t)N;
    const double *p0 = a.pos + sd.off;
    const double *bP = p0 + (size_t)(sd.P - 1) * 3 * NN;
    // blockIdx -> (tile row tr, tile col tc), tc <= tr
    const int b = blockIdx.x;
    int tr = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
    while ((tr + 1) * (tr + 2) / 2 <= b) ++tr;
    while (tr * (tr + 1) / 2 > b) --tr;
    const int tc = b - tr * (tr + 1) / 2;
    const int v0 = tr * TB, u0 = tc * TB, t = threadIdx.x;
    if (t < 3 * TB) {
        const int c = t / TB, i = t % TB;
        rv[c][i] = v0 + i < N ? bP[c * NN + v0 + i] : 0.0;
        ru[c][i] = u0 + i < N ? p0[c * NN + u0 + i] : 0.0;
    }
    __syncthreads();
    const double box = a.box, ib = a.inv_box, k = sd.k;
    // 256 threads: 4 rows at a time, 64 columns
    const int iu = t % TB;
    for (int iv = t / TB; iv < TB; iv += 4) {
        const int v = v0 + iv, u = u0 + iu;
        if (v >= N || u > v) continue;
        const double dx = mimg<BOX>(rv[0][iv] - ru[0][iu], box, ib);
        const double dy = mimg<BOX>(rv[1][iv] - ru[1][iu], box, ib);
        const double dz = mimg<BOX>(rv[2][iv] - ru[2][iu], box, ib);
        const int64_t o = (int64_t)v * (v + 1) / 2 + u;
        if (F32)
            ((float *)dst)[o] = (float)(k * sqlen<true>(dx, dy, dz));
        else
            ((double *)dst)[o] = k * sqlen<false>(dx, dy, dz);
    }
}

hipError_t launch_endpoint_springs(const LaunchArgs &a, int s, int N, int as_float, void *dst, hipStream_t st) {
    const int nt = (N + 63) / 64;
    const int blocks = nt * (nt + 1) / 2;
    const bool box = a.box > 0;
    if (box && as_float)
        hipLaunchKernelGGL((k_endpoint_springs<true, true>), dim3(blocks), dim3(256), 0, st, a, s, dst);
    else if (box)
        hipLaunchKernelGGL((k_endpoint_springs<true, false>), dim3(blocks), dim3(256), 0, st, a, s, dst);
    else if (as_float)
        hipLaunchKernelGGL((k_endpoint_springs<false, true>), dim3(blocks), dim3(256), 0, st, a, s, dst);
    else
        hipLaunchKernelGGL((k_endpoint_springs<false, false>), dim3(blocks), dim3(256), 0, st, a, s, dst);
    return hipGetLastError();
}

} // namespace pimdb
