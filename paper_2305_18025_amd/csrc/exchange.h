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
// 3. Right-looking recursions, blocked.  Thread-owned accumulators: when
//    Z_f[u-1] is known, every accumulator v >= u adds Z_f[u-1] K(u,v), and
//    the owner of v = u then holds Z_f[u] = acc/u.  Steps go in blocks of 64:
//    the wave owning a block's 64 accumulators runs its 64 steps serially
//    with lane broadcasts, while the other waves add the previous block's
//    64 terms to every later accumulator without synchronisation; two
//    workgroup barriers per block.  The backward recursion is the same with rows and columns
//    exchanged; forward and backward run concurrently in separate
//    workgroups.
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
//
// This header holds the fused evaluation kernel (recursions, interior
// springs); exchange_inst.hip instantiates one launch variant of it per
// build job.

#pragma once

#include "common.h"

namespace pimdb {

// ------------------------------------------------------------- recursions
// Both recursions are blocked in BK = 64 steps (one wave's width).  Row j of
// thread t holds accumulator q = j T + t, so block b (accumulators
// [64 b, 64 b + 64)) is row b / W of wave b % W (W = T / 64 waves).
// Forward, iteration k (block k = steps and accumulators [64 k, 64 k + 64)):
//   phase A (all waves): the exponentials of block k's own triangle
//     K(s+1, q+1), s <= q, go to LDS; block k-1's terms for block k's 64
//     accumulators are summed in slices by 4 waves (8 in 16-wave
//     workgroups; partial sums to LDS) while the last wave stages block
//     k+1's endpoints;
//   barrier;
//   phase B: the wave owning block k merges the partial sums and runs the
//     block's 64 steps serially: at step s each lane q >= s adds
//     Z_f[s] K(s+1, q+1) (read from LDS), after which the owner lane q = s
//     holds its final sum and Z_f[s+1] = sum / (s+1) reaches the other lanes
//     by readlane.  Meanwhile every other accumulator beyond block k adds the
//     64 terms of block k-1 (the panel), with no synchronisation;
//   barrier.
// The backward recursion is the mirror image (blocks descending, rows
// q <= s, terms (Z_b[l+1]/l) K(q+1, l)).
//
// Open boundaries in FP64 (DOT): with coordinates taken relative to a
// per-system origin, kappa |a - b|^2 + h = (kappa |a|^2 + h) + kappa |b|^2
// - 2 kappa a.b, so a term's exponent is one add and three FMAs with
// per-row and per-step constants, and the weighted displacements are
// recovered from the weighted step points: sum t (a - b) = a sum t - sum t b.
// The expansion's rounding is about kappa eps |extent|^2 in the exponent
// (1e-12 relative for a cube of side 10).  Periodic systems (the minimum
// image is per pair) and the mixed mode (FP32 pair lengths) keep the direct
// form.
//
// Exponent bookkeeping: an accumulator (A, e) stands for A 2^e; a term
// t 2^te is added as A += t 2^(te - e) while te - e <= RENORM, so A stays
// below 2^(RENORM + 13).  A larger term first moves the reference to
// e = te + RMARGIN (A, W scaled to match), leaving room for later terms up
// to 2^(RENORM + RMARGIN) above it; A stays a normal number (at least
// 2^-RMARGIN times a term), and terms more than 2^114 below the largest
// underflow harmlessly.  In the gauge used here the terms of a row grow
// along the recursion (Z_f gains a link-spring factor per step), so the
// panels take the steps of each block in reverse order, largest first: the
// reference then moves about once per block instead of every few steps.
constexpr int BK = 64;
constexpr int RENORM = 960;
constexpr int RMARGIN = 960;
constexpr int KSPLIT = 8;   // most waves that share the previous block's terms for the diagonal rows
                            // (8 in 16-wave workgroups, else 4)
constexpr int KTRI = BK * (BK + 1) / 2;

// LDS map (doubles):
//   [L_STG, +3*10*BS)  ring of 3 staged blocks, per particle
//                      {x1, y1, z1, xP, yP, zP, h, Df, Db, -}: bead-1 and
//                      bead-P points (relative to the origin in the dot
//                      form), h = -kappa |r^P - r_ref^1|^2, and the dot
//                      form's step constants Df = kappa |r^1|^2,
//                      Db = kappa |r^P|^2 + h
//   [L_ZM, +3*BS)      ring of 3 blocks of broadcast mantissas, per step
//   [L_ZE, +3*BS/2)    matching exponents (ints)
//   [L_ZL, +3*BS)      log2 of the mantissa plus the step's own exponent
//                      constant (what the panel terms use)
// Ring slots hold BS = BK + 2 entries: one guard entry on each side, so a
// panel may read one step past either end of its block without a bounds
// clamp (the guard values are never used).
//   [L_KP, +KTRI)      the diagonal block's exponentials: mantissas,
//                      packed triangle (zero-filled once, so reads past a
//                      row's live part return finite values)
//   [L_KN, +BK*BK/2)   their exponents (ints), full 64 x 64 rows; entries of
//                      lanes a step does not reach hold EMASK (filled once)
//   [L_PA, +KSPLIT*4*BK)  partial sums {A, Wx, Wy, Wz} per wave and lane
//   [L_PE, +KSPLIT*BK/2)  their exponents (ints)
//   [L_DL, +2*L_DLS)   the accumulators a helper delivered for the current
//                      and the next block (split recursions' chain)
//   [L_ABT, +1)        abort flag of a split recursion (int)
//   [L_UR, +2*4*BK)    a helper's urgent-row constants for this and the
//                      next iteration; in a chain, its count of published
//                      steps and the slot waves' count of finished slices
//                      (L_PROG, two ints)
//   [L_UC, +1)         a helper's count of finished urgent slices (int)
//   [LDS_RED, +T)      block reduction scratch of the spring role (a
//                      workgroup runs either a recursion or springs, so
//                      this aliases the recursion regions)
// The chain of a split recursion with a CU of its own also has:
//   [L_KP2, +KTRI), [L_KN2, +BK*BK/2)  a second triangle buffer (the next
//                      block's triangle is formed while the current one is
//                      in use)
constexpr int L_STG = 0;
constexpr int STG = 10; // doubles per staged particle
constexpr int BS = BK + 2;
constexpr int L_ZM = L_STG + 3 * STG * BS;
constexpr int L_ZE = L_ZM + 3 * BS;
constexpr int L_ZL = L_ZE + 3 * BS / 2;
constexpr int L_KP = L_ZL + 3 * BS;
constexpr int L_KN = L_KP + KTRI;
constexpr int L_PA = L_KN + BK * BK / 2;
constexpr int L_PE = L_PA + KSPLIT * 4 * BK;
constexpr int L_DLS = 4 * BK + BK / 2;          // one delivered accumulator {A, Wx, Wy, Wz} x 64 + exponents
constexpr int L_DL = L_PE + KSPLIT * BK / 2;     // two of them (the current and the next block)
constexpr int L_ABT = L_DL + 2 * L_DLS;          // abort flag (int) of a split recursion
constexpr int L_UR = L_ABT + 1;                  // a helper's urgent row constants {px, py, pz, hl} x 64, twice
constexpr int L_UC = L_UR + 2 * 4 * BK;          // a helper's slice counter (int)
constexpr int L_END = L_UC + 1;
constexpr int L_KP2 = L_END;
constexpr int L_KN2 = L_KP2 + KTRI;
constexpr int L_END2 = L_KN2 + BK * BK / 2;
constexpr int L_PROG = L_UR; // a chain's two counters (chains do not use the helpers' urgent rows)
constexpr int LDS_RED = 0;

__device__ __forceinline__ double *stg_block(double *sm, int b) { return sm + L_STG + ((b % 3) * BS + 1) * STG; }
__device__ __forceinline__ double *zm_block(double *sm, int b) { return sm + L_ZM + (b % 3) * BS + 1; }
__device__ __forceinline__ int *ze_block(double *sm, int b) { return (int *)(sm + L_ZE) + (b % 3) * BS + 1; }
__device__ __forceinline__ double *zl_block(double *sm, int b) { return sm + L_ZL + (b % 3) * BS + 1; }
__device__ __forceinline__ int *pe_base(double *sm) { return (int *)(sm + L_PE); }

// Packed triangle of the diagonal block: forward row i_s holds lanes
// [i_s, 64), backward row i_s holds lanes [0, i_s].
template <bool FWD>
__device__ __forceinline__ int tri_index(int is, int lane) {
    return FWD ? is * BK - (is * (is - 1)) / 2 + (lane - is) : (is * (is + 1)) / 2 + lane;
}

__device__ __forceinline__ int add_sat(int a, int b) { return __builtin_elementwise_add_sat(a, b); }
__device__ __forceinline__ int sub_sat(int a, int b) { return __builtin_elementwise_sub_sat(a, b); }

// Accumulator of one row: A 2^e and the term-weighted displacements W 2^e.
struct Acc {
    double A, Wx, Wy, Wz;
    int e;
};

// Move the reference of (A, W) to te + RMARGIN if the term t 2^te is more
// than 2^RENORM above it; returns te - e for the (possibly new) reference.
template <bool WSUM>
__device__ __forceinline__ int acc_shift(Acc &r, int te) {
    int k = sub_sat(te, r.e);
    if (k > RENORM) {
        const int sh = add_sat(k, RMARGIN);
        r.A = ldexp(r.A, -sh);
        if (WSUM) {
            r.Wx = ldexp(r.Wx, -sh);
            r.Wy = ldexp(r.Wy, -sh);
            r.Wz = ldexp(r.Wz, -sh);
        }
        r.e = add_sat(te, RMARGIN);
        k = -RMARGIN;
    }
    return k;
}

template <bool WSUM>
__device__ __forceinline__ void acc_add(Acc &r, double t, int k, double dx, double dy, double dz) {
    const double tn = ldexp(t, k);
    r.A += tn;
    if (WSUM) {
        r.Wx = fma(tn, dx, r.Wx);
        r.Wy = fma(tn, dy, r.Wy);
        r.Wz = fma(tn, dz, r.Wz);
    }
}

// Merge another accumulator into r.
template <bool WSUM>
__device__ __forceinline__ void acc_merge(Acc &r, const Acc &o) {
    const int en = max(r.e, o.e);
    const int a = sub_sat(r.e, en), b = sub_sat(o.e, en);
    r.A = ldexp(r.A, a) + ldexp(o.A, b);
    if (WSUM) {
        r.Wx = ldexp(r.Wx, a) + ldexp(o.Wx, b);
        r.Wy = ldexp(r.Wy, a) + ldexp(o.Wy, b);
        r.Wz = ldexp(r.Wz, a) + ldexp(o.Wz, b);
    }
    r.e = en;
}

// log2(m) for a mantissa m in [0.5, 1): m is scaled into [1/sqrt 2, sqrt 2)
// and ln(m) = 2 atanh(s), s = (m - 1) / (m + 1), |s| <= 0.172, summed as the
// odd series s + s^3/3 + ... + s^21/21 (truncation below 1e-18).
__device__ __forceinline__ double log2_mant(double m) {
    const bool lo = m < 0.70710678118654752;
    const double x = lo ? 2.0 * m : m;
    const double s = (x - 1.0) / (x + 1.0), s2 = s * s;
    double p = 1.0 / 21.0;
#pragma unroll
    for (int k = 9; k >= 0; --k) p = fma(p, s2, 1.0 / (double)(2 * k + 1));
    return (2.0 * LOG2E) * (s * p) - (lo ? 1.0 : 0.0);
}

// K = 2^(kappa |a - b|^2 + h) and the displacement d = a - b (minimum
// image when periodic).
template <bool BOX, bool MIXED>
__device__ __forceinline__ void kterm(double ax, double ay, double az, double bx, double by, double bz, double h,
                                      double kap, double box, double ib, double &p, int &n, double &dx, double &dy,
                                      double &dz) {
    dx = mimg<BOX>(ax - bx, box, ib);
    dy = mimg<BOX>(ay - by, box, ib);
    dz = mimg<BOX>(az - bz, box, ib);
    exp2x(fma(kap, sqlen<MIXED>(dx, dy, dz), h), p, n);
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Accumulator rows of one thread.  Direct form: (px, py, pz) = r_q^P and
// hl = h_q (forward) or (px, py, pz) = r_q^1 (backward).  Dot form:
// (px, py, pz) = -2 kappa times that point, hl = kappa |point|^2 (+ h_q
// forward).  The accumulator's W holds sum t d (direct) or sum t b over the
// step points b (dot).
template <int JJ>
struct Rows {
    double px[JJ], py[JJ], pz[JJ], hl[JJ];
    Acc a[JJ];
};

struct RecCtx {
    double *sm;
    const double *b1, *bP; // bead-1 and bead-P planes of the system
    size_t NN;
    int N, T, t, W, nblk;
    double kap, box, ib;
    double ox, oy, oz; // origin of the dot form (bead 1 of particle 0)
    int32_t *flags;    // status word
    int kp, kn;        // LDS offsets (doubles) of the triangle buffer in use
    int lag;           // split recursions: a helper delivers the block `lag` after the published one
};

// Staged data of one particle.
struct Stage {
    double x1, y1, z1, xP, yP, zP, h, Df, Db;
};

template <bool BOX, bool MIXED>
__device__ __forceinline__ Stage stage_load(const RecCtx &c, int b, bool &bad) {
    constexpr bool DOT = !BOX && !MIXED;
    Stage g{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const int l = b * BK + (c.t & 63);
    if (l < c.N) {
        const size_t NN = c.NN;
        g.x1 = c.b1[l];
        g.y1 = c.b1[NN + l];
        g.z1 = c.b1[2 * NN + l];
        g.xP = c.bP[l];
        g.yP = c.bP[NN + l];
        g.zP = c.bP[2 * NN + l];
        const int r = l < c.N - 1 ? l + 1 : l;
        g.h = -c.kap * sqlen<MIXED>(mimg<BOX>(g.xP - c.b1[r], c.box, c.ib),
                                     mimg<BOX>(g.yP - c.b1[NN + r], c.box, c.ib),
                                     mimg<BOX>(g.zP - c.b1[2 * NN + r], c.box, c.ib));
        bad |= !(g.h <= XHI);
        if (DOT) {
            g.x1 -= c.ox;
            g.y1 -= c.oy;
            g.z1 -= c.oz;
            g.xP -= c.ox;
            g.yP -= c.oy;
            g.zP -= c.oz;
            g.Df = c.kap * (g.x1 * g.x1 + g.y1 * g.y1 + g.z1 * g.z1);
            g.Db = fma(c.kap, g.xP * g.xP + g.yP * g.yP + g.zP * g.zP, g.h);
        }
    }
    return g;
}

__device__ __forceinline__ void stage_store(const RecCtx &c, int b, const Stage &g) {
    double *S = stg_block(c.sm, b) + STG * (c.t & 63);
    S[0] = g.x1;
    S[1] = g.y1;
    S[2] = g.z1;
    S[3] = g.xP;
    S[4] = g.yP;
    S[5] = g.zP;
    S[6] = g.h;
    S[7] = g.Df;
    S[8] = g.Db;
}

// A step's data: forward the bead-1 point of u, backward the bead-P point
// of l; h is h_l (direct form, backward), the step constant Df or Db (dot
// form), else 0.
template <bool FWD, bool DOT>
__device__ __forceinline__ void step_point(const double *S, int i, double &x, double &y, double &z, double &h) {
    const double *u = S + STG * i + (FWD ? 0 : 3);
    x = u[0];
    y = u[1];
    z = u[2];
    h = DOT ? (FWD ? u[7] : u[5]) : (FWD ? 0.0 : u[3]);
}

// The exponent constant of the step whose staged record is su: forward 0
// (direct) or Df (dot); backward h (direct) or Db (dot).
template <bool FWD, bool DOT>
__device__ __forceinline__ double step_const(const double *su) {
    return DOT ? (FWD ? su[7] : su[8]) : (FWD ? 0.0 : su[6]);
}

// Per-row constants of the dot form for the point (x, y, z) (origin
// relative) with h (forward) or 0 (backward).
__device__ __forceinline__ void dot_row(double kap, double x, double y, double z, double h, double &ax, double &ay,
                                        double &az, double &cq) {
    ax = -2.0 * kap * x;
    ay = -2.0 * kap * y;
    az = -2.0 * kap * z;
    cq = fma(kap, x * x + y * y + z * z, h);
}

// Terms of one step for rows [LO, HI), formed in lockstep (each stage of
// the exponential for every row before the next), so the chains of
// different rows interleave.  With 3 or more rows per thread they go in
// groups of 2 (register budget: 3 waves per SIMD).
// Rounding constant of a row with reference exponent e: 1.5 2^52 - e.  For
// |x| < 2^51, t = x + (1.5 2^52 - e) is x rounded to an integer (to nearest
// even, as rint) plus the constant, and the low word of t's bits is
// round(x) - e; so t - constant recovers round(x) exactly, and adding the
// step's exponent ze to the low word gives te - e.  This replaces rint, a
// conversion and a saturating add per term (used where one row per thread
// leaves the registers for the per-row constant).
constexpr double RMAGIC = 6755399441055744.0; // 1.5 2^52
template <int JJ>
__device__ __forceinline__ double row_magic(const Rows<JJ> &R, int j) { return RMAGIC - (double)R.a[j].e; }

template <bool FWD, int LO, int HI, int JJ, bool BOX, bool MIXED, bool WSUM, bool MAG>
__device__ __forceinline__ void panel_step(Rows<JJ> &R, double *Me, const RecCtx &c, double zl, int ze, double ux,
                                           double uy, double uz) {
    constexpr int GM = JJ >= 3 ? 2 : 4;
    if constexpr (HI - LO > GM) {
        panel_step<FWD, LO, LO + GM, JJ, BOX, MIXED, WSUM, MAG>(R, Me, c, zl, ze, ux, uy, uz);
        __builtin_amdgcn_sched_barrier(0);
        panel_step<FWD, LO + GM, HI, JJ, BOX, MIXED, WSUM, MAG>(R, Me, c, zl, ze, ux, uy, uz);
    } else if constexpr (HI > LO) {
        constexpr int G = HI - LO;
        constexpr bool DOT = !BOX && !MIXED;
        double x[G], r[G], f[G], p[G], dx[G], dy[G], dz[G];
        int k[G];
        if (DOT) { // exponent from the row and step constants; W sums t * (step point)
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int j = LO + g;
                x[g] = fma(R.px[j], ux, fma(R.py[j], uy, fma(R.pz[j], uz, R.hl[j] + zl)));
                dx[g] = ux;
                dy[g] = uy;
                dz[g] = uz;
            }
        } else {
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int j = LO + g;
                if (FWD) {
                    dx[g] = mimg<BOX>(R.px[j] - ux, c.box, c.ib);
                    dy[g] = mimg<BOX>(R.py[j] - uy, c.box, c.ib);
                    dz[g] = mimg<BOX>(R.pz[j] - uz, c.box, c.ib);
                } else {
                    dx[g] = mimg<BOX>(ux - R.px[j], c.box, c.ib);
                    dy[g] = mimg<BOX>(uy - R.py[j], c.box, c.ib);
                    dz[g] = mimg<BOX>(uz - R.pz[j], c.box, c.ib);
                }
            }
#pragma unroll
            for (int g = 0; g < G; ++g)
                x[g] = fma(c.kap, sqlen<MIXED>(dx[g], dy[g], dz[g]), FWD ? R.hl[LO + g] + zl : zl);
        }
        // t = x + 1.5 2^52 - e rounds x to an integer (nearest even) and
        // its low word is round(x) - e
        double tm[G];
        if constexpr (MAG) {
#pragma unroll
            for (int g = 0; g < G; ++g) tm[g] = x[g] + Me[LO + g];
#pragma unroll
            for (int g = 0; g < G; ++g) r[g] = tm[g] - Me[LO + g];
        } else {
#pragma unroll
            for (int g = 0; g < G; ++g) r[g] = rint(x[g]);
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            f[g] = x[g] - r[g];
            p[g] = EXP2_C[0];
        }
#pragma unroll
        for (int i = 1; i < EXP2_N; ++i) {
#pragma unroll
            for (int g = 0; g < G; ++g) p[g] = fma(p[g], f[g], EXP2_C[i]);
        }
        bool big = false;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if constexpr (MAG)
                k[g] = (int)(uint32_t)__builtin_bit_cast(uint64_t, tm[g]) + ze;
            else
                k[g] = sub_sat(add_sat(ze, (int)r[g]), R.a[LO + g].e);
            big |= k[g] > RENORM;
        }
        // wave-uniform and rare (steps go largest first): a real branch, so
        // the common path carries none of the rescaling instructions
        if (__builtin_expect(__builtin_amdgcn_ballot_w64(big) != 0, 0)) {
#pragma unroll
            for (int g = 0; g < G; ++g) {
                k[g] = acc_shift<WSUM>(R.a[LO + g], add_sat(ze, (int)r[g]));
                if constexpr (MAG) Me[LO + g] = row_magic(R, LO + g);
            }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) acc_add<WSUM>(R.a[LO + g], p[g], k[g], dx[g], dy[g], dz[g]);
    }
}

// Two steps' terms for one row (row J): both exponentials are formed in one
// stretch of code, so their dependency chains overlap where a single row
// would leave the wave waiting on each FMA in turn; they are then added in
// the order of two single steps (the reference moves, when one is needed,
// happen exactly as they would step by step, so the result is the same).
template <bool FWD, int J, int JJ, bool BOX, bool MIXED, bool WSUM, bool MAG>
__device__ __forceinline__ void panel_step2(Rows<JJ> &R, double *Me, const RecCtx &c, double zl0, int ze0,
                                            double ux0, double uy0, double uz0, double zl1, int ze1, double ux1,
                                            double uy1, double uz1) {
    constexpr bool DOT = !BOX && !MIXED;
    const double zl[2] = {zl0, zl1}, ux[2] = {ux0, ux1}, uy[2] = {uy0, uy1}, uz[2] = {uz0, uz1};
    const int ze[2] = {ze0, ze1};
    double x[2], r[2], f[2], p[2], dx[2], dy[2], dz[2], tm[2];
    int k[2];
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        if (DOT) {
            x[g] = fma(R.px[J], ux[g], fma(R.py[J], uy[g], fma(R.pz[J], uz[g], R.hl[J] + zl[g])));
            dx[g] = ux[g];
            dy[g] = uy[g];
            dz[g] = uz[g];
        } else {
            if (FWD) {
                dx[g] = mimg<BOX>(R.px[J] - ux[g], c.box, c.ib);
                dy[g] = mimg<BOX>(R.py[J] - uy[g], c.box, c.ib);
                dz[g] = mimg<BOX>(R.pz[J] - uz[g], c.box, c.ib);
            } else {
                dx[g] = mimg<BOX>(ux[g] - R.px[J], c.box, c.ib);
                dy[g] = mimg<BOX>(uy[g] - R.py[J], c.box, c.ib);
                dz[g] = mimg<BOX>(uz[g] - R.pz[J], c.box, c.ib);
            }
            x[g] = fma(c.kap, sqlen<MIXED>(dx[g], dy[g], dz[g]), FWD ? R.hl[J] + zl[g] : zl[g]);
        }
    }
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        if constexpr (MAG) {
            tm[g] = x[g] + Me[J];
            r[g] = tm[g] - Me[J];
        } else {
            r[g] = rint(x[g]);
        }
        f[g] = x[g] - r[g];
        p[g] = EXP2_C[0];
    }
#pragma unroll
    for (int i = 1; i < EXP2_N; ++i) {
#pragma unroll
        for (int g = 0; g < 2; ++g) p[g] = fma(p[g], f[g], EXP2_C[i]);
    }
    bool big = false;
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        if constexpr (MAG)
            k[g] = (int)(uint32_t)__builtin_bit_cast(uint64_t, tm[g]) + ze[g];
        else
            k[g] = sub_sat(add_sat(ze[g], (int)r[g]), R.a[J].e);
        big |= k[g] > RENORM;
    }
    if (__builtin_expect(__builtin_amdgcn_ballot_w64(big) != 0, 0)) {
        // step by step: the second term's exponent is taken relative to the
        // reference the first one may have moved
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            const int kk = acc_shift<WSUM>(R.a[J], add_sat(ze[g], (int)r[g]));
            if constexpr (MAG) Me[J] = row_magic(R, J);
            acc_add<WSUM>(R.a[J], p[g], kk, dx[g], dy[g], dz[g]);
        }
    } else {
        acc_add<WSUM>(R.a[J], p[0], k[0], dx[0], dy[0], dz[0]);
        acc_add<WSUM>(R.a[J], p[1], k[1], dx[1], dy[1], dz[1]);
    }
}

// Panel: rows [LO, HI) add the terms of the steps of block blk.  Full
// blocks in the 1- and 2-row kernels run an unrolled loop; otherwise steps
// go in pairs with two alternating sets of step values, each read one step
// ahead, so no values are copied between iterations.
template <bool FWD, int LO, int HI, int JJ, bool BOX, bool MIXED, bool WSUM, bool UNR, bool MAG>
__device__ __forceinline__ void panel(Rows<JJ> &R, const RecCtx &c, int blk) {
    if constexpr (HI > LO) {
        constexpr bool DOT = !BOX && !MIXED;
        const int nst = min(BK, c.N - blk * BK);
        const double *S = stg_block(c.sm, blk);
        const double *Z = zl_block(c.sm, blk);
        const int *E = ze_block(c.sm, blk);
        // the block's steps from the last of the recursion's order to the
        // first (largest terms first); -1 .. BK: guard entries at the ends
        auto at = [&](int n) { return FWD ? nst - 1 - n : n; };
        double Me[JJ];
        if constexpr (MAG) Me[0] = row_magic(R, 0);
        if constexpr (UNR) {
            if (nst == BK) {
                // full block (1- and 2-row kernels): no tail test, four steps
                // per loop trip with immediate LDS offsets
                if constexpr (HI - LO == 1) { // one row: steps in pairs
#pragma unroll 2
                    for (int n = 0; n < BK; n += 2) {
                        const int i0 = FWD ? BK - 1 - n : n, i1 = FWD ? BK - 2 - n : n + 1;
                        double ax, ay, az, ah, bx, by, bz, bh;
                        step_point<FWD, DOT>(S, i0, ax, ay, az, ah);
                        step_point<FWD, DOT>(S, i1, bx, by, bz, bh);
                        panel_step2<FWD, LO, JJ, BOX, MIXED, WSUM, MAG>(R, Me, c, Z[i0], E[i0], ax, ay, az, Z[i1],
                                                                        E[i1], bx, by, bz);
                    }
                } else {
#pragma unroll 4
                    for (int n = 0; n < BK; ++n) {
                        const int ii = FWD ? BK - 1 - n : n;
                        double ux, uy, uz, uh;
                        step_point<FWD, DOT>(S, ii, ux, uy, uz, uh);
                        panel_step<FWD, LO, HI, JJ, BOX, MIXED, WSUM, MAG>(R, Me, c, Z[ii], E[ii], ux, uy, uz);
                    }
                }
                return;
            }
        }
        double ax, ay, az, ah, bx, by, bz, bh, za, zb;
        int ea, eb;
        int i = at(0);
        step_point<FWD, DOT>(S, i, ax, ay, az, ah);
        za = Z[i];
        ea = E[i];
        for (int n = 0; n < nst; n += 2) {
            i = at(n + 1);
            step_point<FWD, DOT>(S, i, bx, by, bz, bh);
            zb = Z[i];
            eb = E[i];
            if constexpr (HI - LO == 1) { // one row: both steps' terms together
                if (n + 1 < nst) {
                    panel_step2<FWD, LO, JJ, BOX, MIXED, WSUM, MAG>(R, Me, c, za, ea, ax, ay, az, zb, eb, bx, by, bz);
                    i = at(n + 2);
                    step_point<FWD, DOT>(S, i, ax, ay, az, ah);
                    za = Z[i];
                    ea = E[i];
                } else {
                    panel_step<FWD, LO, HI, JJ, BOX, MIXED, WSUM, MAG>(R, Me, c, za, ea, ax, ay, az);
                }
                continue;
            }
            panel_step<FWD, LO, HI, JJ, BOX, MIXED, WSUM, MAG>(R, Me, c, za, ea, ax, ay, az);
            if (n + 1 < nst) {
                i = at(n + 2);
                step_point<FWD, DOT>(S, i, ax, ay, az, ah);
                za = Z[i];
                ea = E[i];
                panel_step<FWD, LO, HI, JJ, BOX, MIXED, WSUM, MAG>(R, Me, c, zb, eb, bx, by, bz);
            }
        }
    }
}

// Phase A1: exponentials of block k's triangle into LDS, 2080 entries in 33
// folded rows of 64 lanes: work row wr < 32 takes (wr, c) for lanes c >= wr
// and (63 - wr, 63 - c) for c < wr; work row 32 takes the diagonal entries
// of rows 32..63.  (Coordinates of the forward triangle s <= q; the
// backward one is its mirror image.)  Wave w takes work rows w, w + W, ...
// (or, given w0 >= 0, work rows w0, w0 + ws, ...).
template <bool FWD, bool BOX, bool MIXED>
__device__ __forceinline__ void diag_terms(const RecCtx &c, int k, int w0 = -1, int ws = 0) {
    const int lane = c.t & 63;
    const int nst = min(BK, c.N - k * BK);
    const double *S = stg_block(c.sm, k);
    double *KP = c.sm + c.kp;
    int *KN = (int *)(c.sm + c.kn);
    if (w0 < 0) {
        w0 = c.t >> 6;
        ws = c.W;
    }
    for (int wr = w0; wr <= BK / 2; wr += ws) {
        int r, q; // forward-triangle row (step) and column (accumulator)
        bool ok = true;
        if (wr < BK / 2) {
            r = lane >= wr ? wr : BK - 1 - wr;
            q = lane >= wr ? lane : BK - 1 - lane;
        } else {
            ok = lane < BK / 2;
            r = q = BK - 1 - lane;
        }
        const int is = FWD ? r : BK - 1 - r;  // step
        const int iq = FWD ? q : BK - 1 - q;  // accumulator
        if (ok && is < nst) {
            const double *me = S + STG * iq;
            double ux, uy, uz, uh, p, dx, dy, dz;
            int n;
            step_point<FWD, false>(S, is, ux, uy, uz, uh);
            if (FWD)
                kterm<BOX, MIXED>(me[3], me[4], me[5], ux, uy, uz, me[6], c.kap, c.box, c.ib, p, n, dx, dy, dz);
            else
                kterm<BOX, MIXED>(ux, uy, uz, me[0], me[1], me[2], uh, c.kap, c.box, c.ib, p, n, dx, dy, dz);
            KP[tri_index<FWD>(is, iq)] = p;
            KN[is * BK + iq] = n;
        }
    }
}

// Phase A2: wave w < KSPLIT sums the terms of its slice of block prev's
// steps for block k's accumulators (lane i: 64 k + i) into LDS.
// Waves that share the previous block's terms for the diagonal rows: 8 in
// 16-wave workgroups, else up to 4 (the other waves run panels).
__device__ __forceinline__ int partial_waves(const RecCtx &c) { return c.W >= 16 ? KSPLIT : min(KSPLIT / 2, c.W); }

// Steps [i0, i1) of block blk (counted largest term first, as in the
// panels) added to row 0 of R.  ILP2: the steps in pairs whose
// exponentials overlap (the same sums).
template <bool FWD, bool BOX, bool MIXED, bool WSUM, bool MAG, bool ILP2>
__device__ __forceinline__ void slice_sum(Rows<1> &R, const RecCtx &c, int blk, int i0, int i1) {
    const int nst = min(BK, c.N - blk * BK);
    const double *S = stg_block(c.sm, blk);
    const double *Z = zl_block(c.sm, blk);
    const int *E = ze_block(c.sm, blk);
    double Me[1] = {row_magic(R, 0)};
    int n = i0;
    if constexpr (ILP2) {
        for (; n + 1 < i1; n += 2) {
            const int ia = FWD ? nst - 1 - n : n;
            const int ib = FWD ? nst - 2 - n : n + 1;
            double ax, ay, az, ah, bx, by, bz, bh;
            step_point<FWD, !BOX && !MIXED>(S, ia, ax, ay, az, ah);
            step_point<FWD, !BOX && !MIXED>(S, ib, bx, by, bz, bh);
            panel_step2<FWD, 0, 1, BOX, MIXED, WSUM, MAG>(R, Me, c, Z[ia], E[ia], ax, ay, az, Z[ib], E[ib], bx, by,
                                                         bz);
        }
    }
    for (; n < i1; ++n) {
        const int i = FWD ? nst - 1 - n : n;
        double ux, uy, uz, uh;
        step_point<FWD, !BOX && !MIXED>(S, i, ux, uy, uz, uh);
        panel_step<FWD, 0, 1, 1, BOX, MIXED, WSUM, MAG>(R, Me, c, Z[i], E[i], ux, uy, uz);
    }
}

// A partial sum {A, W} to partial-sum slot `slot` of LDS (lane i: row i).
__device__ __forceinline__ void write_partial(const RecCtx &c, int slot, const Acc &r) {
    const int lane = c.t & 63;
    double *PA = c.sm + L_PA + slot * 4 * BK + lane;
    PA[0] = r.A;
    PA[BK] = r.Wx;
    PA[2 * BK] = r.Wy;
    PA[3 * BK] = r.Wz;
    pe_base(c.sm)[slot * BK + lane] = r.e;
}

__device__ __forceinline__ Acc read_partial(const RecCtx &c, int slot) {
    const int lane = c.t & 63;
    const double *PA = c.sm + L_PA + slot * 4 * BK + lane;
    return Acc{PA[0], PA[BK], PA[2 * BK], PA[3 * BK], pe_base(c.sm)[slot * BK + lane]};
}

// The row of accumulator 64 k + lane (from the staged block k) in the form
// the terms use, with an empty accumulator.
template <bool FWD, bool BOX, bool MIXED>
__device__ __forceinline__ Rows<1> staged_row(const RecCtx &c, int k) {
    const double *me = stg_block(c.sm, k) + STG * (c.t & 63);
    Rows<1> R;
    if (FWD) {
        R.px[0] = me[3];
        R.py[0] = me[4];
        R.pz[0] = me[5];
        R.hl[0] = me[6];
    } else {
        R.px[0] = me[0];
        R.py[0] = me[1];
        R.pz[0] = me[2];
        R.hl[0] = 0.0;
    }
    if (!BOX && !MIXED) dot_row(c.kap, R.px[0], R.py[0], R.pz[0], R.hl[0], R.px[0], R.py[0], R.pz[0], R.hl[0]);
    R.a[0] = Acc{0.0, 0.0, 0.0, 0.0, EMIN};
    return R;
}

// Phase A2 for block k: wave w < ns adds its slice of block prev's steps
// for block k's accumulators (rows from the staged block k) into LDS slot w.
template <bool FWD, bool BOX, bool MIXED, bool WSUM, bool MAG, bool ILP2 = false>
__device__ __forceinline__ void diag_partial(const RecCtx &c, int k, int prev, int ns) {
    const int w = c.t >> 6;
    if (w >= ns) return;
    Rows<1> R = staged_row<FWD, BOX, MIXED>(c, k);
    const int nst = min(BK, c.N - prev * BK); // previous block: full except the backward top
    slice_sum<FWD, BOX, MIXED, WSUM, MAG, ILP2>(R, c, prev, (nst * w) / ns, (nst * (w + 1)) / ns);
    write_partial(c, w, R.a[0]);
}

// Phase B, owner wave: merge the partial sums, then run block k's steps
// serially on row j (lane i: accumulator 64 k + i).  Afterwards every lane's
// row is final: its published value goes to the broadcast ring for the
// panels and its results to global memory.
// PROG: the broadcast ring's values go out every eight steps (each lane's
// current value; those of the lanes already final are what the ring
// needs), followed by the count of steps done, pbase + steps, in the LDS
// word *prog; the log2 form of the ring is then left to its readers.
template <bool FWD, int j, int JJ, bool BOX, bool MIXED, bool WSUM, bool UNR, bool PROG = false>
__device__ __forceinline__ void diagonal(Rows<JJ> &R, const RecCtx &c, int k, bool has_prev, double *zm_out,
                                         double *ze_out, double *r_out, int ns, int *prog = nullptr,
                                         int pbase = 0) {
    const int lane = c.t & 63, q = k * BK + lane, N = c.N;
    const size_t NN = c.NN;
    const int nst = min(BK, N - k * BK);
    Acc &r = R.a[j];
    if (has_prev) {
        // the partial sums join in one pass: the largest reference first,
        // then each sum rescaled to it and added in slot order (the same
        // sums as merging them one by one); when the partial sums all hold
        // that reference they are added as they are.  The reads go in
        // batches (all exponents, then four slots at a time) so that their
        // latencies overlap; slots past ns are read (they lie inside the
        // partial-sum region) but not used.
        const int *PE = pe_base(c.sm) + lane;
        int pe[KSPLIT];
#pragma unroll
        for (int w = 0; w < KSPLIT; ++w) pe[w] = PE[w * BK];
        __builtin_amdgcn_sched_barrier(0);
        int en = r.e;
#pragma unroll
        for (int w = 0; w < KSPLIT; ++w)
            if (w < ns) en = max(en, pe[w]);
        bool same = true;
#pragma unroll
        for (int w = 0; w < KSPLIT; ++w)
            if (w < ns) same &= pe[w] == en;
        const bool one_ref = __builtin_amdgcn_ballot_w64(!same) == 0;
        const int a0 = sub_sat(r.e, en);
        r.A = ldexp(r.A, a0);
        if (WSUM) {
            r.Wx = ldexp(r.Wx, a0);
            r.Wy = ldexp(r.Wy, a0);
            r.Wz = ldexp(r.Wz, a0);
        }
#pragma unroll
        for (int h = 0; h < KSPLIT; h += 4) {
            double pa[4][4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const double *PA = c.sm + L_PA + (h + u) * 4 * BK + lane;
                pa[u][0] = PA[0];
                if (WSUM) {
                    pa[u][1] = PA[BK];
                    pa[u][2] = PA[2 * BK];
                    pa[u][3] = PA[3 * BK];
                }
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (h + u < ns) {
                    const int b = one_ref ? 0 : sub_sat(pe[h + u], en);
                    r.A += ldexp(pa[u][0], b);
                    if (WSUM) {
                        r.Wx += ldexp(pa[u][1], b);
                        r.Wy += ldexp(pa[u][2], b);
                        r.Wz += ldexp(pa[u][3], b);
                    }
                }
            }
        }
        r.e = en;
    }
    const double ivd = FWD ? 1.0 / (double)(q + 1) : (q > 0 ? 1.0 / (double)q : 0.0);
    const double *S = stg_block(c.sm, k);
    const double *KPl = c.sm + c.kp + lane;
    const int *KNl = (const int *)(c.sm + c.kn) + lane;
    const int first = FWD ? 0 : nst - 1;
    double zm = zm_block(c.sm, k)[first];
    int ze = ze_block(c.sm, k)[first];
    // PROG: this lane's ring entry (the step that reads its value), if any
    const int psp = FWD ? q + 1 : q - 1;
    const bool pown = PROG && q < N && psp >= 0 && psp < N;
    double *pzm = PROG ? zm_block(c.sm, max(psp, 0) / BK) + max(psp, 0) % BK : nullptr;
    int *pze = PROG ? ze_block(c.sm, max(psp, 0) / BK) + max(psp, 0) % BK : nullptr;
    double lmz = 0.0; // this lane's current value (mantissa, exponent)
    int lez = 0;
    auto publish = [&](int done) {
        if (pown) {
            *pzm = lmz;
            *pze = lez;
        }
        // LDS requests of a wave complete in order: the values are in place
        // before the count that announces them
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        if (lane == 0) __hip_atomic_store(prog, pbase + done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    // One step: every lane adds the term of step is (lanes the step does not
    // reach read an EMASK exponent and add nothing; their KP reads stay
    // inside the zero-filled triangle), then the owner (lane is) is complete
    // and its scaled sum is broadcast.
    auto step = [&](int is, double p, int n, double x, double y, double z) {
        double dx = 0.0, dy = 0.0, dz = 0.0;
        if (WSUM) {
            if (!BOX && !MIXED) {
                dx = x;
                dy = y;
                dz = z;
            } else if (FWD) {
                dx = mimg<BOX>(R.px[j] - x, c.box, c.ib);
                dy = mimg<BOX>(R.py[j] - y, c.box, c.ib);
                dz = mimg<BOX>(R.pz[j] - z, c.box, c.ib);
            } else {
                dx = mimg<BOX>(x - R.px[j], c.box, c.ib);
                dy = mimg<BOX>(y - R.py[j], c.box, c.ib);
                dz = mimg<BOX>(z - R.pz[j], c.box, c.ib);
            }
        }
        const int te = add_sat(ze, n);
        int kk = sub_sat(te, r.e);
        if (__builtin_expect(__builtin_amdgcn_ballot_w64(kk > RENORM) != 0, 0)) kk = acc_shift<WSUM>(r, te);
        acc_add<WSUM>(r, zm * p, kk, dx, dy, dz);
        const double zz = r.A * ivd;
        lmz = __builtin_amdgcn_frexp_mant(zz);
        lez = r.e + __builtin_amdgcn_frexp_exp(zz);
        zm = readlane_f64(lmz, is);
        ze = __builtin_amdgcn_readlane(lez, is);
    };
    bool done = false;
    if constexpr (UNR) {
        if (nst == BK) {
            // full block: unrolled, so every LDS offset is an immediate and
            // the serial chain carries no address arithmetic; each step's
            // values are read before the previous step's chain runs
            double xs[2], ys[2], zs[2], ps[2], uh;
            int es[2];
            {
                const int is = FWD ? 0 : BK - 1;
                step_point<FWD, !BOX && !MIXED>(S, is, xs[0], ys[0], zs[0], uh);
                ps[0] = KPl[tri_index<FWD>(is, 0)];
                es[0] = KNl[is * BK];
            }
#pragma unroll
            for (int i = 0; i < BK; ++i) {
                const int is = FWD ? i : BK - 1 - i;
                const int cu = i & 1, nx = cu ^ 1;
                if (i + 1 < BK) {
                    const int is2 = FWD ? i + 1 : BK - 2 - i;
                    step_point<FWD, !BOX && !MIXED>(S, is2, xs[nx], ys[nx], zs[nx], uh);
                    ps[nx] = KPl[tri_index<FWD>(is2, 0)];
                    es[nx] = KNl[is2 * BK];
                }
                step(is, ps[cu], es[cu], xs[cu], ys[cu], zs[cu]);
                if constexpr (PROG) {
                    if ((i & 7) == 7) publish(i + 1);
                }
            }
            done = true;
        }
    }
    if (!done) {
        // partial blocks (and the wider kernels, to bound code size): a
        // step's values are read one step ahead so the LDS latency stays
        // off the serial chain
        struct DStep {
            double p, x, y, z;
            int n;
        };
        auto fetch = [&](int i) {
            const int is = FWD ? min(i, nst - 1) : max(nst - 1 - i, 0);
            DStep d;
            d.p = KPl[tri_index<FWD>(is, 0)];
            d.n = KNl[is * BK];
            double uh;
            step_point<FWD, !BOX && !MIXED>(S, is, d.x, d.y, d.z, uh);
            return d;
        };
        DStep da = fetch(0), db;
        for (int i = 0; i < nst; i += 2) {
            db = fetch(i + 1);
            step(FWD ? i : nst - 1 - i, da.p, da.n, da.x, da.y, da.z);
            if (PROG && ((i & 7) == 7 || i + 1 == nst)) publish(i + 1);
            if (i + 1 < nst) {
                da = fetch(i + 2);
                step(FWD ? i + 1 : nst - 2 - i, db.p, db.n, db.x, db.y, db.z);
                if (PROG && ((i & 7) == 6 || i + 2 == nst)) publish(i + 2);
            }
        }
    }
    if (q < N) {
        const double zz = r.A * ivd;
        const double mz = __builtin_amdgcn_frexp_mant(zz);
        const int ez = r.e + __builtin_amdgcn_frexp_exp(zz);
        // the open-chain gauge carries the chain's cumulative spring
        // exponents; beyond 2^29 binary orders they would approach the
        // empty-accumulator sentinel, so the input is out of range
        if (__builtin_expect(ez > EZ_LIM || ez < -EZ_LIM, 0)) set_flag(c.flags, ST_RANGE);
        const int sp = FWD ? q + 1 : q - 1; // step that reads this value
        if (!PROG && sp >= 0 && sp < N) {
            const double *su = stg_block(c.sm, sp / BK) + STG * (sp % BK);
            zm_block(c.sm, sp / BK)[sp % BK] = mz;
            ze_block(c.sm, sp / BK)[sp % BK] = ez;
            zl_block(c.sm, sp / BK)[sp % BK] = log2_mant(mz) + step_const<FWD, !BOX && !MIXED>(su);
        }
        if (FWD) { // Z_f[q+1]
            zm_out[q + 1] = mz;
            ze_out[q + 1] = (double)ez;
        } else { // Z_b[q+1]
            zm_out[q + 1] = __builtin_amdgcn_frexp_mant(r.A);
            ze_out[q + 1] = (double)(r.e + __builtin_amdgcn_frexp_exp(r.A));
        }
        if (WSUM) {
            const double ia = 1.0 / r.A;
            double mx = r.Wx * ia, my = r.Wy * ia, mz2 = r.Wz * ia;
            if (!BOX && !MIXED) { // from the weighted mean step point
                const double *me = S + STG * lane + (FWD ? 3 : 0);
                const double sg = FWD ? -1.0 : 1.0;
                mx = fma(sg, mx, FWD ? me[0] : -me[0]);
                my = fma(sg, my, FWD ? me[1] : -me[1]);
                mz2 = fma(sg, mz2, FWD ? me[2] : -me[2]);
            }
            r_out[q] = mx;
            r_out[NN + q] = my;
            r_out[2 * NN + q] = mz2;
        }
    }
}

// Phase B of one wave.  Forward: live rows [LO, JJ) (blocks >= k);
// backward: live rows [0, HI) (blocks <= k).  DG: this wave owns block k
// (row LO forward, row HI-1 backward).
template <bool FWD, int LO, int HI, bool DG, int JJ, bool BOX, bool MIXED, bool WSUM, bool UNR, bool MAG>
__device__ __forceinline__ void wave_iter(Rows<JJ> &R, const RecCtx &c, int k, double *zm_out, double *ze_out,
                                          double *r_out) {
    const int prev = FWD ? k - 1 : k + 1;
    const bool has_prev = FWD ? k > 0 : k + 1 < c.nblk;
    if constexpr (DG) {
        constexpr int jd = FWD ? LO : HI - 1;
        // the serial chain is the critical path of phase B: its wave issues
        // first whenever it is ready
        __builtin_amdgcn_s_setprio(2);
        diagonal<FWD, jd, JJ, BOX, MIXED, WSUM, UNR>(R, c, k, has_prev, zm_out, ze_out, r_out, partial_waves(c));
        __builtin_amdgcn_s_setprio(0);
        if (has_prev) {
            if (FWD)
                panel<FWD, LO + 1, HI, JJ, BOX, MIXED, WSUM, UNR, MAG>(R, c, prev);
            else
                panel<FWD, LO, HI - 1, JJ, BOX, MIXED, WSUM, UNR, MAG>(R, c, prev);
        }
    } else {
        if (has_prev) panel<FWD, LO, HI, JJ, BOX, MIXED, WSUM, UNR, MAG>(R, c, prev);
    }
}

// Runtime (first live row / number of live rows, owner?) -> compiled variant.
template <bool FWD, int X, int JJ, bool BOX, bool MIXED, bool WSUM, bool UNR, bool MAG>
__device__ __forceinline__ void wave_dispatch(Rows<JJ> &R, const RecCtx &c, int k, int x, bool dg, double *zm_out,
                                              double *ze_out, double *r_out) {
    if constexpr (X <= JJ) {
        if (x == X) {
            if (FWD) {
                if constexpr (X < JJ) {
                    if (dg)
                        wave_iter<FWD, X, JJ, true, JJ, BOX, MIXED, WSUM, UNR, MAG>(R, c, k, zm_out, ze_out, r_out);
                    else
                        wave_iter<FWD, X, JJ, false, JJ, BOX, MIXED, WSUM, UNR, MAG>(R, c, k, zm_out, ze_out, r_out);
                }
            } else {
                if constexpr (X > 0) {
                    if (dg)
                        wave_iter<FWD, 0, X, true, JJ, BOX, MIXED, WSUM, UNR, MAG>(R, c, k, zm_out, ze_out, r_out);
                    else
                        wave_iter<FWD, 0, X, false, JJ, BOX, MIXED, WSUM, UNR, MAG>(R, c, k, zm_out, ze_out, r_out);
                }
            }
        } else {
            wave_dispatch<FWD, X + 1, JJ, BOX, MIXED, WSUM, UNR, MAG>(R, c, k, x, dg, zm_out, ze_out, r_out);
        }
    }
}

// Where a recursion writes its results: the forward Z_f, Z_b mantissas and
// exponents and the weighted mean displacements (workspace, or the adjoint
// state when the forward half saves them).
template <bool FWD>
__device__ __forceinline__ void rec_outputs(const LaunchArgs &a, const SysDesc &sd, double *&zm_out, double *&ze_out,
                                            double *&r_out) {
    const int N = sd.N;
    if (FWD) {
        double *base = (a.mode & M_SAVE) ? a.state + sd.st : a.ws + sd.ws;
        zm_out = base + ((a.mode & M_SAVE) ? StLayout::zf_m(N) : WsLayout::zf_m(N));
        ze_out = base + ((a.mode & M_SAVE) ? StLayout::zf_e(N) : WsLayout::zf_e(N));
        r_out = base + ((a.mode & M_SAVE) ? StLayout::rf(N) : WsLayout::rf(N));
    } else {
        double *base = a.ws + sd.ws;
        zm_out = base + WsLayout::zb_m(N);
        ze_out = base + WsLayout::zb_e(N);
        r_out = base + WsLayout::rb(N);
    }
}

// Row j of R holds accumulator q (0 <= q < N, or an unused row): its point
// (forward bead P of q with h_q, backward bead 1 of q) in the form the
// terms use, and an empty accumulator.
template <bool FWD, int JJ, bool BOX, bool MIXED>
__device__ __forceinline__ void load_row(Rows<JJ> &R, int j, const RecCtx &c, int q, bool &range_bad) {
    const int N = c.N;
    const size_t NN = c.NN;
    R.px[j] = R.py[j] = R.pz[j] = R.hl[j] = 0.0;
    if (q >= 0 && q < N) {
        if (FWD) {
            R.px[j] = c.bP[q];
            R.py[j] = c.bP[NN + q];
            R.pz[j] = c.bP[2 * NN + q];
            const int r = q < N - 1 ? q + 1 : q;
            R.hl[j] = -c.kap * sqlen<MIXED>(mimg<BOX>(R.px[j] - c.b1[r], c.box, c.ib),
                                             mimg<BOX>(R.py[j] - c.b1[NN + r], c.box, c.ib),
                                             mimg<BOX>(R.pz[j] - c.b1[2 * NN + r], c.box, c.ib));
            range_bad |= !(R.hl[j] <= XHI);
        } else {
            R.px[j] = c.b1[q];
            R.py[j] = c.b1[NN + q];
            R.pz[j] = c.b1[2 * NN + q];
        }
        if (!BOX && !MIXED)
            dot_row(c.kap, R.px[j] - c.ox, R.py[j] - c.oy, R.pz[j] - c.oz, R.hl[j], R.px[j], R.py[j], R.pz[j],
                    R.hl[j]);
    }
    R.a[j] = Acc{0.0, 0.0, 0.0, 0.0, EMIN};
}

// Before the first block of a serial recursion: stage the first block,
// publish the first broadcast value (Z_f[0] = 1 since V^[1,0] = 0, or
// Z_b[N+1] / N = 1 / N), write the fixed ends of the outputs and fill the
// diagonal triangle's LDS (see the LDS map).  Ends with a barrier.
template <bool FWD, bool BOX, bool MIXED>
__device__ __forceinline__ void rec_prologue(const RecCtx &c, double *zm_out, double *ze_out, bool &range_bad) {
    const int t = c.t, T = c.T, N = c.N, w = t >> 6, nblk = c.nblk;
    const int b0 = FWD ? 0 : nblk - 1;
    const int s0 = FWD ? 0 : N - 1;
    if (w == 0) {
        const Stage g = stage_load<BOX, MIXED>(c, b0, range_bad);
        stage_store(c, b0, g);
        if ((t & 63) == s0 % BK) {
            const double z0 = FWD ? 1.0 : 1.0 / (double)N;
            const double m0 = __builtin_amdgcn_frexp_mant(z0);
            constexpr bool DOT = !BOX && !MIXED;
            zm_block(c.sm, b0)[s0 % BK] = m0;
            ze_block(c.sm, b0)[s0 % BK] = __builtin_amdgcn_frexp_exp(z0);
            zl_block(c.sm, b0)[s0 % BK] = log2_mant(m0) + (DOT ? (FWD ? g.Df : g.Db) : (FWD ? 0.0 : g.h));
        }
    }
    if (t == 0) {
        if (FWD) {
            zm_out[0] = 1.0;
            ze_out[0] = 0.0;
        } else {
            zm_out[N + 1] = 1.0;
            ze_out[N + 1] = 0.0;
        }
    }
    for (int i = t; i < BK * BK; i += T) ((int *)(c.sm + c.kn))[i] = EMASK;
    for (int i = t; i < KTRI; i += T) c.sm[c.kp + i] = 0.0;
    // loads of the rows are complete before the loop (a wait inside it would
    // also wait for the staging loads issued there)
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}

template <bool FWD, int JJ, bool BOX, bool MIXED, bool WSUM, bool UNR, bool MAG>
__device__ __forceinline__ void recursion_rows(const LaunchArgs &a, const SysDesc &sd, const RecCtx &c) {
    const int t = c.t, T = c.T, W = c.W, w = t >> 6, nblk = c.nblk;
    double *zm_out, *ze_out, *r_out;
    rec_outputs<FWD>(a, sd, zm_out, ze_out, r_out);
    Rows<JJ> R;
    bool range_bad = false;
#pragma unroll
    for (int j = 0; j < JJ; ++j) load_row<FWD, JJ, BOX, MIXED>(R, j, c, j * T + t, range_bad);
    rec_prologue<FWD, BOX, MIXED>(c, zm_out, ze_out, range_bad);
    for (int it = 0; it < nblk; ++it) {
        const int k = FWD ? it : nblk - 1 - it;
        const int prev = FWD ? k - 1 : k + 1;
        const bool has_prev = FWD ? k > 0 : k + 1 < nblk;
        // phase A; the next block is staged by the last wave (its loads are
        // issued first and land in LDS before the barrier; its ring slot last
        // held block k-2, which is no longer read)
        const int nb = FWD ? k + 1 : k - 1;
        const bool stage = w == W - 1 && nb >= 0 && nb < nblk;
        Stage g{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (stage) g = stage_load<BOX, MIXED>(c, nb, range_bad);
        diag_terms<FWD, BOX, MIXED>(c, k);
        if (has_prev) { // the longest work of phase A
            __builtin_amdgcn_s_setprio(1);
            diag_partial<FWD, BOX, MIXED, WSUM, MAG>(c, k, prev, partial_waves(c));
            __builtin_amdgcn_s_setprio(0);
        }
        if (stage) stage_store(c, nb, g);
        lds_barrier();
        // phase B
        int x;
        bool dg;
        if (FWD) { // first row j with j W + w >= k
            x = k <= w ? 0 : (k - w + W - 1) / W;
            dg = x * W + w == k;
        } else { // number of rows j with j W + w <= k
            x = k < w ? 0 : min((k - w) / W + 1, JJ);
            dg = x > 0 && (x - 1) * W + w == k;
        }
        wave_dispatch<FWD, 0, JJ, BOX, MIXED, WSUM, UNR, MAG>(R, c, k, x, dg, zm_out, ze_out, r_out);
        lds_barrier();
    }
    if (range_bad) set_flag(a.flags, ST_RANGE);
}


// ------------------------------------------------------- split recursions
// For small batches one workgroup per recursion leaves most CUs idle, so a
// system's recursion may be spread over 1 + H workgroups (nhelp = H), with
// a lag L (2, or 3 when every workgroup has a CU of its own):
//  - the chain workgroup adds the terms of the L - 1 blocks before block k
//    to block k's accumulators, forms the triangle's exponentials, runs the
//    block's serial steps, and publishes the block's step values (what the
//    panels use) to the exchange area;
//  - helper h owns the accumulators of every H-th block from L + h up
//    (forward; backward from nblk - 1 - L - h down).  For every published
//    block i it adds block i's terms to its accumulators of blocks at least
//    L blocks further in recursion order, and the accumulator of the block
//    exactly L further then holds every term but those of the L - 1 blocks
//    before it (which the chain adds): it is delivered to the chain.
// A delivery for block k is made while the chain runs block k - L + 1 or
// later, so the hand-over latency stays off the serial path.  The chain
// forms the terms of the L - 1 blocks before block k while the steps of
// block k-1 run (chain_rows_prog).  Flags and payloads are
// device-scope relaxed atomics, which bypass the caches that are not
// coherent across the XCDs without flushing them; a producer waits for its
// payload stores to complete before it stores the flag.  Every wait is
// bounded in time: on expiry it sets ST_TIMEOUT and the workgroup returns.
// The host keeps a split launch within the workgroups that are resident at
// once, so no wait depends on a workgroup that has not started.

__device__ __forceinline__ void st_dev(double *p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(int *p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_dev(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_dev(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One wave spins until *flag is set; false (and ST_TIMEOUT) after `ticks`
// of the 100 MHz constant clock.
__device__ __forceinline__ bool wave_wait(const int *flag, int32_t *status, uint64_t ticks) {
    const uint64_t t0 = wall_clock64();
    while (__builtin_amdgcn_readfirstlane(ld_dev(flag)) == 0) {
        __builtin_amdgcn_s_sleep(1);
        if (wall_clock64() - t0 > ticks) {
            if ((threadIdx.x & 63) == 0) set_flag(status, ST_TIMEOUT);
            return false;
        }
    }
    return true;
}

// A delivered accumulator {A, Wx, Wy, Wz} x 64 and its exponents, from the
// exchange area into LDS (D): every load is issued before the first store,
// so their latencies overlap (an atomic load is not moved past the stores
// that follow it).
__device__ __forceinline__ void fetch_delivery(double *D, const double *src, const int *esrc, int lane) {
    const double a0 = ld_dev(src + lane), a1 = ld_dev(src + BK + lane), a2 = ld_dev(src + 2 * BK + lane),
                 a3 = ld_dev(src + 3 * BK + lane);
    const int e = ld_dev(esrc + lane);
    D[lane] = a0;
    D[BK + lane] = a1;
    D[2 * BK + lane] = a2;
    D[3 * BK + lane] = a3;
    ((int *)(D + 4 * BK))[lane] = e;
}

// After the wave's payload stores: wait for them, then set the flag.
__device__ __forceinline__ void wave_signal(int *flag) {
    __builtin_amdgcn_s_waitcnt(0);
    if ((threadIdx.x & 63) == 0) st_dev(flag, 1);
}

struct XsPtrs {
    double *pub_zl;
    int *pub_ze;
    double *del_acc;
    int *del_e;
    int *pub_flag, *del_flag;
};

template <bool FWD>
__device__ __forceinline__ XsPtrs xs_ptrs(const LaunchArgs &a, const SysDesc &sd, int nblk) {
    const int d = FWD ? 0 : 1;
    double *x = a.ws + sd.xs;
    int *fl = (int *)(x + XsLayout::flags(nblk));
    return XsPtrs{x + XsLayout::pub_zl(nblk, d), (int *)(x + XsLayout::pub_ze(nblk, d)),
                  x + XsLayout::del_acc(nblk, d), (int *)(x + XsLayout::del_e(nblk, d)),
                  fl + (2 * d) * nblk, fl + (2 * d + 1) * nblk};
}

// log2 form of block blk's broadcast values for its steps n0 .. n1 - 1
// (counted largest term first): log2 of the mantissa plus the step's own
// exponent constant, one step per lane, into the LDS ring (what the panel
// terms use).
template <bool FWD, bool BOX, bool MIXED>
__device__ __forceinline__ void ring_log2(const RecCtx &c, int blk, int n0, int n1) {
    const int l = c.t & 63;
    const int nst = min(BK, c.N - blk * BK);
    if (n0 + l < n1) {
        const int i = FWD ? nst - 1 - (n0 + l) : n0 + l;
        zl_block(c.sm, blk)[i] =
            log2_mant(zm_block(c.sm, blk)[i]) + step_const<FWD, !BOX && !MIXED>(stg_block(c.sm, blk) + STG * i);
    }
}

// Chain workgroup of a split recursion: 16 waves with a CU of its own and
// lag 3 (DBUF: a second triangle buffer in LDS), or 8 waves sharing a CU
// and lag 2.  While wave 0 merges block k's partial sums and delivery and
// runs its steps,
//  - slot waves (none on wave 0's SIMD when waves go to SIMDs in turn) each
//    form block k+1's partial sum over their eighths of the block's steps:
//    with lag 3 first the terms of block k-1's slice (its values are
//    known); then, in the dot form, the terms of block k's slice without
//    their Z factor, and, as wave 0 publishes the values (eight steps at a
//    time), the products with them; otherwise the whole terms follow the
//    published values;
//  - with DBUF, three waves form block k+1's triangle in the other buffer
//    (else all waves form it after the steps, before a second barrier);
//  - the last wave publishes block k-1's step values for the helpers,
//    fetches block k+1's delivery and stages block k+2 (into the ring slot
//    of block k-1 once the slot waves are done with it).
// So the serial path carries the steps, the merge and one barrier (two
// without DBUF).
constexpr int WIDE_SLOTS = 8, WIDE_TRI = 3;
// Slot waves (none on wave 0's SIMD when waves go to SIMDs in turn): the
// first of the eight slices of wave w (-1: none); a slot wave takes every
// fourth slice from there in 8-wave workgroups (one slice in 16-wave ones).
__device__ __forceinline__ int prog_slot(int w, int W) {
    if (W >= 16) return ((w & 3) != 0 && w < 11) ? w - 1 - (w >> 2) : -1;
    return (w >= 1 && w <= 3) ? w - 1 : (w == 5 ? 3 : -1);
}
__device__ __forceinline__ int wide_tri(int w) { return w == 11 ? 0 : (w == 13 || w == 14 ? w - 12 : -1); }
constexpr int YC = BK / WIDE_SLOTS; // steps of a full slice

// Spin (one wave) until the LDS word *cnt reaches target; bounded like
// the waits between workgroups (ST_TIMEOUT after `ticks`, and the wave goes
// on with whatever the word announces).
__device__ __forceinline__ void lds_wait(const int *cnt, int target, int32_t *status, uint64_t ticks) {
    const uint64_t t0 = wall_clock64();
    while (__builtin_amdgcn_readfirstlane(__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) <
           target) {
        __builtin_amdgcn_s_sleep(1);
        if (wall_clock64() - t0 > ticks) {
            if ((threadIdx.x & 63) == 0) set_flag(status, ST_TIMEOUT);
            break;
        }
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

template <bool FWD, bool BOX, bool MIXED, bool WSUM, bool DBUF>
__device__ __forceinline__ void chain_rows_prog(const LaunchArgs &a, const SysDesc &sd, const RecCtx &c) {
    constexpr bool DOT = !BOX && !MIXED;
    const int t = c.t, W = c.W, w = t >> 6, lane = t & 63, nblk = c.nblk, lag = c.lag;
    constexpr int sls = DBUF ? WIDE_SLOTS : WIDE_SLOTS / 2; // slices per slot wave: one (DBUF) or two
    const int sl0 = prog_slot(w, DBUF ? 16 : 8), tr = DBUF ? wide_tri(w) : -1;
    const bool last = w == W - 1;
    double *zm_out, *ze_out, *r_out;
    rec_outputs<FWD>(a, sd, zm_out, ze_out, r_out);
    const XsPtrs X = xs_ptrs<FWD>(a, sd, nblk);
    int *abort_flag = (int *)(c.sm + L_ABT);
    int *prog = (int *)(c.sm + L_PROG), *xdone = prog + 1;
    if (t == 0) {
        *abort_flag = 0;
        *prog = 0;
        *xdone = 0;
    }
    bool range_bad = false;
    RecCtx c2 = c; // the second triangle buffer (DBUF)
    if (DBUF) {
        c2.kp = L_KP2;
        c2.kn = L_KN2;
        for (int i = t; i < BK * BK; i += c.T) ((int *)(c.sm + L_KN2))[i] = EMASK;
        for (int i = t; i < KTRI; i += c.T) c.sm[L_KP2 + i] = 0.0;
    }
    const int first = FWD ? 0 : nblk - 1;
    const int di = FWD ? 1 : -1;
    Stage g{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (last) g = stage_load<BOX, MIXED>(c, first + di, range_bad);
    rec_prologue<FWD, BOX, MIXED>(c, zm_out, ze_out, range_bad);
    diag_terms<FWD, BOX, MIXED>(c, first);
    if (last) stage_store(c, first + di, g);
    lds_barrier();
    for (int it = 0; it < nblk; ++it) {
        const int k = first + di * it;
        const int prev = k - di, nb = k + di, nn = k + 2 * di;
        const bool has_prev = it > 0, has_nb = it + 1 < nblk;
        const RecCtx &ck = (DBUF && (it & 1)) ? c2 : c; // block k's triangle
        const RecCtx &cn = (DBUF && !(it & 1)) ? c2 : c; // block k+1's
        if (!DBUF && it > 0) { // one buffer: block k's triangle once block k-1's steps are done
            diag_terms<FWD, BOX, MIXED>(c, k);
            lds_barrier();
        }
        if (w == 0) { // the serial steps
            Rows<1> R = staged_row<FWD, BOX, MIXED>(c, k);
            const bool delivered = FWD ? k >= lag : k <= nblk - 1 - lag;
            if (delivered) {
                const double *D = c.sm + L_DL + (it & 1) * L_DLS;
                R.a[0] = Acc{D[lane], D[BK + lane], D[2 * BK + lane], D[3 * BK + lane], ((const int *)(D + 4 * BK))[lane]};
            }
            __builtin_amdgcn_s_setprio(2);
            diagonal<FWD, 0, 1, BOX, MIXED, WSUM, true, true>(R, ck, k, has_prev, zm_out, ze_out, r_out, WIDE_SLOTS,
                                                              prog, it * BK);
            __builtin_amdgcn_s_setprio(0);
            // wave 0 holds no staged data: assigned here, its registers
            // are free during the steps
            g = Stage{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        } else if (sl0 >= 0) {
            if (has_nb) {
#pragma unroll
                for (int sx = 0; sx < WIDE_SLOTS / sls; ++sx) {
                    const int sl = sl0 + sx * sls;
                    Rows<1> R = staged_row<FWD, BOX, MIXED>(c, nb);
                    if (lag >= 3 && has_prev) { // block k-1's terms (its values are known)
                        const int np = min(BK, c.N - prev * BK);
                        const int n0 = np - (np * (sl + 1)) / WIDE_SLOTS, n1 = np - (np * sl) / WIDE_SLOTS;
                        ring_log2<FWD, BOX, MIXED>(c, prev, n0, n1);
                        slice_sum<FWD, BOX, MIXED, WSUM, false, true>(R, c, prev, n0, n1);
                    }
                    if (sx + 1 == WIDE_SLOTS / sls) { // the wave's last slice
                        // (its reads are issued before the count: LDS
                        // requests of a wave complete in order)
                        __atomic_signal_fence(__ATOMIC_SEQ_CST);
                        if (lane == 0)
                            __hip_atomic_fetch_add(xdone, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                    // block k's slice: chain positions [i0, i1), i.e. steps
                    // n0 .. n1 - 1 counted largest term first
                    const int nst = min(BK, c.N - k * BK);
                    const int i0 = (nst * sl) / WIDE_SLOTS, i1 = (nst * (sl + 1)) / WIDE_SLOTS;
                    const int n0 = nst - i1, n1 = nst - i0;
                    if (DOT) {
                        if (i1 - i0 == YC) {
                            const double *S = stg_block(c.sm, k);
                            double yp[YC];
                            int yn[YC];
#pragma unroll
                            for (int m = 0; m < YC; ++m) { // the terms without their Z factor, four at a time
                                const int i = FWD ? i0 + m : nst - 1 - (i0 + m);
                                double ux, uy, uz, uh;
                                step_point<FWD, true>(S, i, ux, uy, uz, uh);
                                exp2x(fma(R.px[0], ux, fma(R.py[0], uy, fma(R.pz[0], uz, R.hl[0] + uh))), yp[m], yn[m]);
                                if (m == YC / 2 - 1) __builtin_amdgcn_sched_barrier(0);
                            }
                            lds_wait(prog, it * BK + i1, a.flags, a.wait_ticks);
                            const double *Zm = zm_block(c.sm, k);
                            const int *Ze = ze_block(c.sm, k);
                            double zv[YC];
                            int te[YC];
                            int mx = 0;
#pragma unroll
                            for (int m = 0; m < YC; ++m) {
                                const int i = FWD ? i0 + m : nst - 1 - (i0 + m);
                                zv[m] = Zm[i];
                                te[m] = Ze[i];
                            }
                            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                            for (int m = 0; m < YC; ++m) {
                                te[m] = add_sat(yn[m], te[m]);
                                mx = m == 0 ? te[0] : max(mx, te[m]);
                            }
                            // one reference move at most, for the slice's largest
                            // term (moving it at the first such term gives the
                            // same sums)
                            Acc &r = R.a[0];
                            if (__builtin_expect(__builtin_amdgcn_ballot_w64(sub_sat(mx, r.e) > RENORM) != 0, 0))
                                acc_shift<WSUM>(r, mx);
#pragma unroll
                            for (int m = YC - 1; m >= 0; --m) { // largest term first
                                const int i = FWD ? i0 + m : nst - 1 - (i0 + m);
                                double ux, uy, uz, uh;
                                step_point<FWD, true>(S, i, ux, uy, uz, uh);
                                acc_add<WSUM>(r, yp[m] * zv[m], sub_sat(te[m], r.e), ux, uy, uz);
                            }
                        } else {
                            lds_wait(prog, it * BK + max(i1, 1), a.flags, a.wait_ticks);
                            ring_log2<FWD, BOX, MIXED>(c, k, n0, n1);
                            slice_sum<FWD, BOX, MIXED, WSUM, false, false>(R, c, k, n0, n1);
                        }
                    } else {
                        lds_wait(prog, it * BK + max(i1, 1), a.flags, a.wait_ticks);
                        ring_log2<FWD, BOX, MIXED>(c, k, n0, n1);
                        slice_sum<FWD, BOX, MIXED, WSUM, false, true>(R, c, k, n0, n1);
                    }
                    write_partial(c, sl, R.a[0]);
                }
            } else if (lane == 0) {
                __hip_atomic_fetch_add(xdone, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        } else {
            if (last && has_prev) { // block k-1's step values for the helpers, first
                const int np = min(BK, c.N - prev * BK);
                const int i = lane < np ? lane : np - 1;
                const double zl = log2_mant(zm_block(c.sm, prev)[i]) +
                                  step_const<FWD, DOT>(stg_block(c.sm, prev) + STG * i);
                st_dev(X.pub_zl + (size_t)prev * BK + lane, zl);
                st_dev(X.pub_ze + (size_t)prev * BK + lane, ze_block(c.sm, prev)[lane]);
            }
            // block k+2's loads overlap the wait for the published stores
            if (last && it + 2 < nblk) g = stage_load<BOX, MIXED>(c, nn, range_bad);
            if (last && has_prev) wave_signal(X.pub_flag + prev);
            if (last && has_nb) { // block k+1's delivery
                const bool dl = FWD ? nb >= lag : nb <= nblk - 1 - lag;
                if (dl) {
                    if (wave_wait(X.del_flag + nb, a.flags, a.wait_ticks))
                        fetch_delivery(c.sm + L_DL + ((it + 1) & 1) * L_DLS, X.del_acc + (size_t)nb * 4 * BK,
                                       X.del_e + (size_t)nb * BK, lane);
                    else if (lane == 0)
                        *abort_flag = 1;
                }
            }
            if (DBUF && has_nb && tr >= 0) diag_terms<FWD, BOX, MIXED>(cn, nb, tr, WIDE_TRI);
            if (last && it + 2 < nblk) {
                // block k+2 goes to block k-1's ring slot once the slot
                // waves have read block k-1
                lds_wait(xdone, sls * (it + 1), a.flags, a.wait_ticks);
                stage_store(c, nn, g);
            }
        }
        lds_barrier();
        if (*abort_flag) return;
    }
    if (last) { // the last block (no helper needs it; published for completeness)
        const int kl = first + di * (nblk - 1);
        const int np = min(BK, c.N - kl * BK);
        const int i = lane < np ? lane : np - 1;
        const double zl =
            log2_mant(zm_block(c.sm, kl)[i]) + step_const<FWD, DOT>(stg_block(c.sm, kl) + STG * i);
        st_dev(X.pub_zl + (size_t)kl * BK + lane, zl);
        st_dev(X.pub_ze + (size_t)kl * BK + lane, ze_block(c.sm, kl)[lane]);
        wave_signal(X.pub_flag + kl);
    }
    if (range_bad) set_flag(a.flags, ST_RANGE);
}

// Helper blocks, ascending: b(m) = b0 + m H for m < nown (forward b0 =
// lag + h; backward every H-th block from nblk - 1 - lag - h down to the
// smallest, b0).
__device__ __forceinline__ void helper_blocks(bool fwd, int nblk, int H, int h, int lag, int &b0, int &nown) {
    if (fwd) {
        b0 = lag + h;
        nown = b0 < nblk ? (nblk - 1 - b0) / H + 1 : 0;
    } else {
        const int top = nblk - 1 - lag - h;
        b0 = top >= 0 ? top % H : 0;
        nown = top >= 0 ? (top - b0) / H + 1 : 0;
    }
}

// One wave's work on published block i: the panel over its live rows.
// URG: this wave holds the block `lag` further in recursion order (row LO
// forward, HI - 1 backward), whose terms of block i the first nslices row
// waves have summed in slices (LDS slots 0 .. nslices-1); once all slices
// are in, this wave merges them into the row and delivers it, then runs its
// other rows.
template <bool FWD, int LO, int HI, bool URG, int JJ, bool BOX, bool MIXED, bool WSUM, bool UNR, bool MAG>
__device__ __forceinline__ void helper_iter(Rows<JJ> &R, const RecCtx &c, int i, const XsPtrs &X, int nslices,
                                            int target) {
    if constexpr (URG) {
        constexpr int ju = FWD ? LO : HI - 1;
        const int lane = c.t & 63;
        // the other row waves count their finished slices in LDS
        const int *cnt = (const int *)(c.sm + L_UC);
        while (__builtin_amdgcn_readfirstlane(__hip_atomic_load(cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP)) <
               target)
            __builtin_amdgcn_s_sleep(1);
        Acc r = R.a[ju];
        for (int sl = 0; sl < nslices; ++sl) acc_merge<WSUM>(r, read_partial(c, sl));
        const int b = FWD ? i + c.lag : i - c.lag;
        double *dst = X.del_acc + (size_t)b * 4 * BK + lane;
        st_dev(dst, r.A);
        st_dev(dst + BK, r.Wx);
        st_dev(dst + 2 * BK, r.Wy);
        st_dev(dst + 3 * BK, r.Wz);
        st_dev(X.del_e + (size_t)b * BK + lane, r.e);
        wave_signal(X.del_flag + b);
        if (FWD)
            panel<FWD, LO + 1, HI, JJ, BOX, MIXED, WSUM, UNR, MAG>(R, c, i);
        else
            panel<FWD, LO, HI - 1, JJ, BOX, MIXED, WSUM, UNR, MAG>(R, c, i);
    } else {
        panel<FWD, LO, HI, JJ, BOX, MIXED, WSUM, UNR, MAG>(R, c, i);
    }
}

template <bool FWD, int X_, int JJ, bool BOX, bool MIXED, bool WSUM, bool UNR, bool MAG>
__device__ __forceinline__ void helper_dispatch(Rows<JJ> &R, const RecCtx &c, int i, int x, bool urg,
                                                const XsPtrs &X, int nslices, int target) {
    if constexpr (X_ <= JJ) {
        if (x == X_) {
            if (FWD) {
                if constexpr (X_ < JJ) {
                    if (urg)
                        helper_iter<FWD, X_, JJ, true, JJ, BOX, MIXED, WSUM, UNR, MAG>(R, c, i, X, nslices, target);
                    else
                        helper_iter<FWD, X_, JJ, false, JJ, BOX, MIXED, WSUM, UNR, MAG>(R, c, i, X, nslices, target);
                }
            } else {
                if constexpr (X_ > 0) {
                    if (urg)
                        helper_iter<FWD, 0, X_, true, JJ, BOX, MIXED, WSUM, UNR, MAG>(R, c, i, X, nslices, target);
                    else
                        helper_iter<FWD, 0, X_, false, JJ, BOX, MIXED, WSUM, UNR, MAG>(R, c, i, X, nslices, target);
                }
            }
        } else {
            helper_dispatch<FWD, X_ + 1, JJ, BOX, MIXED, WSUM, UNR, MAG>(R, c, i, x, urg, X, nslices, target);
        }
    }
}

// The fetch wave of a helper (its last wave, which holds no rows) copies
// published block i into the LDS ring: its points (loaded before the flag
// is seen) and its step values; and, when that iteration has a block to
// deliver (ub >= 0), that block's row constants into urgent slot us.  False
// after a wait timed out.
template <bool FWD, bool BOX, bool MIXED>
__device__ __forceinline__ bool helper_fetch(const LaunchArgs &a, const RecCtx &c, const XsPtrs &X, int i, int ub,
                                             int us) {
    const int lane = c.t & 63;
    bool unused = false;
    const Stage g = stage_load<BOX, MIXED>(c, i, unused);
    if (ub >= 0) {
        Rows<1> U;
        load_row<FWD, 1, BOX, MIXED>(U, 0, c, ub * BK + lane, unused);
        double *D = c.sm + L_UR + us * 4 * BK + lane;
        D[0] = U.px[0];
        D[BK] = U.py[0];
        D[2 * BK] = U.pz[0];
        D[3 * BK] = U.hl[0];
    }
    if (!wave_wait(X.pub_flag + i, a.flags, a.wait_ticks)) return false;
    const double zl = ld_dev(X.pub_zl + (size_t)i * BK + lane); // both loads before the stores
    const int ze = ld_dev(X.pub_ze + (size_t)i * BK + lane);
    zl_block(c.sm, i)[lane] = zl;
    ze_block(c.sm, i)[lane] = ze;
    stage_store(c, i, g);
    return true;
}

// Helper h of a split recursion: row j of wave w < WR holds its block
// b(j WR + w), with WR row waves chosen by the host (four, one per SIMD,
// when the helper has a CU of its own; otherwise all but the last wave);
// the last wave fetches the published blocks one ahead of the panels, so
// the wait and the loads overlap the arithmetic.
template <bool FWD, int JJ, bool BOX, bool MIXED, bool WSUM, bool UNR, bool MAG>
__device__ __forceinline__ void helper_rows(const LaunchArgs &a, const SysDesc &sd, const RecCtx &c, int h) {
    const int t = c.t, w = t >> 6, lane = t & 63, nblk = c.nblk, H = sd.nhelp;
    const int WR = min(c.W - 1, a.help_rows); // row waves
    const int nsl = min(WR, KSPLIT);          // of which the first nsl slice the urgent row (LDS slots)
    const int lag = c.lag;
    int b0, nown;
    helper_blocks(FWD, nblk, H, h, lag, b0, nown);
    if (nown == 0) return;
    const XsPtrs X = xs_ptrs<FWD>(a, sd, nblk);
    int *abort_flag = (int *)(c.sm + L_ABT);
    Rows<JJ> R;
    bool range_bad = false;
#pragma unroll
    for (int j = 0; j < JJ; ++j) {
        const int m = j * WR + w;
        load_row<FWD, JJ, BOX, MIXED>(R, j, c, (w < WR && m < nown) ? (b0 + m * H) * BK + lane : -1, range_bad);
    }
    // published blocks that some row still needs, in recursion order
    const int blast = b0 + (nown - 1) * H;
    const int i_begin = FWD ? 0 : nblk - 1;
    const int i_end = FWD ? blast - lag : b0 + lag; // inclusive
    const int di = FWD ? 1 : -1;
    // the block this helper delivers after block i (-1: none)
    auto urgent_block = [&](int i) {
        const int ub = FWD ? i + lag : i - lag;
        return (ub >= b0 && ub <= blast && (ub - b0) % H == 0) ? ub : -1;
    };
    int *cnt = (int *)(c.sm + L_UC);
    if (t == 0) {
        *abort_flag = 0;
        *cnt = 0;
    }
    __syncthreads();
    const int wf = c.W - 1; // the fetch wave; waves WR .. wf-1 only keep the barriers
    if (w == wf && !helper_fetch<FWD, BOX, MIXED>(a, c, X, i_begin, urgent_block(i_begin), 0) && lane == 0)
        *abort_flag = 1;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    int nurg = 0; // urgent iterations so far
    for (int i = i_begin, it = 0; FWD ? i <= i_end : i >= i_end; i += di, ++it) {
        if (*abort_flag) return;
        const int ub = urgent_block(i);
        if (ub >= 0) ++nurg;
        if (w == wf) {
            if (i != i_end && !helper_fetch<FWD, BOX, MIXED>(a, c, X, i + di, urgent_block(i + di), (it + 1) & 1) &&
                lane == 0)
                *abort_flag = 1;
        } else if (w < WR) {
            if (ub >= 0 && w < nsl) { // this wave's slice of block i's terms for the urgent row
                const double *D = c.sm + L_UR + (it & 1) * 4 * BK + lane;
                Rows<1> U;
                U.px[0] = D[0];
                U.py[0] = D[BK];
                U.pz[0] = D[2 * BK];
                U.hl[0] = D[3 * BK];
                U.a[0] = Acc{0.0, 0.0, 0.0, 0.0, EMIN};
                const int nst = min(BK, c.N - i * BK);
                slice_sum<FWD, BOX, MIXED, WSUM, false, true>(U, c, i, (nst * w) / nsl, (nst * (w + 1)) / nsl);
                write_partial(c, w, U.a[0]);
            }
            int x;
            bool urg;
            if (FWD) { // live: blocks >= i + lag, i.e. m >= m0
                const int m0 = i <= h ? 0 : (i - h + H - 1) / H;
                x = m0 <= w ? 0 : (m0 - w + WR - 1) / WR;
                urg = ub >= 0 && x * WR + w == m0;
            } else { // live: blocks <= i - lag, i.e. m < L
                const int L = i - lag >= b0 ? min((i - lag - b0) / H + 1, nown) : 0;
                x = L - 1 >= w ? min((L - 1 - w) / WR + 1, JJ) : 0;
                urg = ub >= 0 && x > 0 && (x - 1) * WR + w == L - 1;
            }
            // count this wave's finished slice for the urgent row's owner (one
            // lane: a per-lane operand would be reduced by a scalar loop first)
            if (ub >= 0 && w < nsl && lane == 0)
                __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
            helper_dispatch<FWD, 0, JJ, BOX, MIXED, WSUM, UNR, MAG>(R, c, i, x, urg, X, nsl, nurg * nsl);
        }
        lds_barrier();
    }
    if (range_bad) set_flag(a.flags, ST_RANGE);
}

// Dispatch on the number of rows the system needs, JJ = ceil(N / T) <= J,
// so that no thread carries rows past the end of a smaller system.
// The one-row kernels round term exponents with the row constant (MAG)
// when the system is narrow enough for the low word not to wrap (wrap_ok),
// else with the saturating sequence.
template <int JJ, int J, bool FWD, bool BOX, bool MIXED, bool WSUM>
__device__ __forceinline__ void rec_dispatch(const LaunchArgs &a, const SysDesc &sd, const RecCtx &c, int jj,
                                             bool wrap_ok) {
    if constexpr (JJ <= J) {
        if (jj == JJ) {
            if constexpr (J == 1) {
                if (wrap_ok)
                    recursion_rows<FWD, JJ, BOX, MIXED, WSUM, true, true>(a, sd, c);
                else
                    recursion_rows<FWD, JJ, BOX, MIXED, WSUM, true, false>(a, sd, c);
            } else {
                recursion_rows<FWD, JJ, BOX, MIXED, WSUM, (J <= 2), false>(a, sd, c);
            }
        } else {
            rec_dispatch<JJ + 1, J, FWD, BOX, MIXED, WSUM>(a, sd, c, jj, wrap_ok);
        }
    }
}

// Helpers: JJ = rows per thread the helper needs (its blocks over the waves).
template <int JJ, int J, bool FWD, bool BOX, bool MIXED, bool WSUM>
__device__ __forceinline__ void help_dispatch(const LaunchArgs &a, const SysDesc &sd, const RecCtx &c, int h, int jj,
                                              bool wrap_ok) {
    if constexpr (JJ <= J) {
        if (jj == JJ) {
            if constexpr (J == 1) {
                if (wrap_ok)
                    helper_rows<FWD, JJ, BOX, MIXED, WSUM, true, true>(a, sd, c, h);
                else
                    helper_rows<FWD, JJ, BOX, MIXED, WSUM, true, false>(a, sd, c, h);
            } else {
                helper_rows<FWD, JJ, BOX, MIXED, WSUM, (J <= 2), false>(a, sd, c, h);
            }
        } else {
            help_dispatch<JJ + 1, J, FWD, BOX, MIXED, WSUM>(a, sd, c, h, jj, wrap_ok);
        }
    }
}

// Largest squared distance of a bead-1 point and of a bead-P point from the
// origin (bead 1 of particle 0), over the whole system; every thread gets
// the maxima.  Uses LDS slots of the partial-sum region, which the
// recursion first writes two barriers later.
__device__ __forceinline__ void system_extent(const RecCtx &c, double &r1, double &rP) {
    const size_t NN = c.NN;
    double m1 = 0.0, mP = 0.0;
    for (int q = c.t; q < c.N; q += c.T) {
        const double x1 = c.b1[q] - c.ox, y1 = c.b1[NN + q] - c.oy, z1 = c.b1[2 * NN + q] - c.oz;
        const double xP = c.bP[q] - c.ox, yP = c.bP[NN + q] - c.oy, zP = c.bP[2 * NN + q] - c.oz;
        m1 = fmax(m1, x1 * x1 + y1 * y1 + z1 * z1);
        mP = fmax(mP, xP * xP + yP * yP + zP * zP);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        m1 = fmax(m1, __shfl_xor(m1, o));
        mP = fmax(mP, __shfl_xor(mP, o));
    }
    double *slot = c.sm + L_PA;
    const int w = c.t >> 6;
    if ((c.t & 63) == 0) {
        slot[2 * w] = m1;
        slot[2 * w + 1] = mP;
    }
    __syncthreads();
    r1 = 0.0;
    rP = 0.0;
    for (int i = 0; i < c.W; ++i) {
        r1 = fmax(r1, slot[2 * i]);
        rP = fmax(rP, slot[2 * i + 1]);
    }
}

// A recursion workgroup: the whole recursion (nhelp = 0), the chain of a
// split recursion (helper < 0), or helper `helper` of one.  WIDE: split
// launches whose workgroups each have a CU (lag 3).
template <int J, bool FWD, bool BOX, bool MIXED, bool WSUM, bool SPLIT, bool WIDE>
__device__ __forceinline__ void recursion_role(const LaunchArgs &a, const SysDesc sd, double *sm, int helper) {
    RecCtx c;
    c.sm = sm;
    c.NN = (size_t)sd.N;
    c.b1 = a.pos + sd.off;
    c.bP = a.pos + sd.off + (size_t)(sd.P - 1) * 3 * c.NN;
    c.N = sd.N;
    c.T = blockDim.x;
    c.t = threadIdx.x;
    c.W = c.T / 64;
    c.nblk = (sd.N + BK - 1) / BK;
    c.kap = sd.kappa;
    c.box = a.box;
    c.ib = a.inv_box;
    c.ox = c.b1[0];
    c.oy = c.b1[c.NN];
    c.oz = c.b1[2 * c.NN];
    c.flags = a.flags;
    c.kp = L_KP;
    c.kn = L_KN;
    c.lag = WIDE ? 3 : 2;
    // Range checks on the system's extent D (largest bead-P to bead-1
    // distance, at most the sum of the two radii about the origin; with
    // the minimum image at most sqrt(3) L / 2):
    //  - a term's exponent relative to its row's reference stays inside
    //    +-2^31 when |kappa| D^2 <= 2^30 (term exponents are at least
    //    kappa D^2 - 1, references at most about 2^29 + 2^28 unless the
    //    range flag is set), which the row-constant rounding needs;
    //  - the open FP64 dot form rounds about eps |kappa| |p - o|^2 in each
    //    exponent: past DOT_LIM the 1e-10 accuracy is no longer assured,
    //    which the status word reports (the direct form has no such limit).
    double r1, rP;
    system_extent(c, r1, rP);
    double D = sqrt(r1) + sqrt(rP);
    if (BOX && a.box > 0) D = fmin(D, 0.8660254037844387 * a.box);
    const bool wrap_ok = -sd.kappa * D * D <= 1073741824.0; // 2^30
    if (!BOX && !MIXED && c.t == 0 && -sd.kappa * fmax(r1, rP) > DOT_LIM) set_flag(a.flags, ST_PRECISION);
    if constexpr (SPLIT) {
        if (sd.nhelp > 0 && helper < 0) {
            chain_rows_prog<FWD, BOX, MIXED, WSUM, WIDE>(a, sd, c);
            return;
        }
        if (sd.nhelp > 0) {
            int b0, nown;
            helper_blocks(FWD, c.nblk, sd.nhelp, helper, c.lag, b0, nown);
            const int wr = min(c.W - 1, a.help_rows);
            const int jj = max(1, (nown + wr - 1) / wr); // rows on the row waves
            help_dispatch<1, J, FWD, BOX, MIXED, WSUM>(a, sd, c, helper, jj, wrap_ok);
            return;
        }
    }
    const int jj = (sd.N + c.T - 1) / c.T;
    rec_dispatch<1, J, FWD, BOX, MIXED, WSUM>(a, sd, c, jj, wrap_ok);
}

// ---------------------------------------------------------------- springs
// One thread per particle, loop over beads.  Interior energies E_int(l)
// (Theory, "Reducing the potential", interior springs j = 1..P-1), interior
// bead forces -m w_P^2 (2 r^j - r^{j+1} - r^{j-1}) for j = 2..P-1 (Theory,
// "Force on interior beads"), and the optional trap.  In distinguishable mode
// every ring closes on itself and all beads are written here.
template <bool BOX, int GB>
__device__ __forceinline__ void springs_role(const LaunchArgs &a, const SysDesc sd, int si, int chunk, double *sm) {
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
        // positions and forces never alias (part of the interface), so the
        // loads of later beads may be issued ahead of this bead's stores
        const double *__restrict__ p0 = a.pos + sd.off + q;
        double *__restrict__ fo = wf ? a.out + sd.off + q : nullptr;
        double cx = p0[0], cy = p0[NN], cz = p0[2 * NN];
        double vx, vy, vz; // previous bead
        if (dist) {
            const size_t o = (size_t)(P - 1) * 3 * NN;
            vx = p0[o];
            vy = p0[o + NN];
            vz = p0[o + 2 * NN];
        } else {
            vx = cx; vy = cy; vz = cz;
        }
        double ei = 0.0, et = 0.0;
        // beads in groups of GB: the group's loads are all issued before any
        // of its arithmetic, so the memory latency is paid once per group
        for (int j0 = 0; j0 < P; j0 += GB) {
            double gx[GB], gy[GB], gz[GB];
#pragma unroll
            for (int u = 0; u < GB; ++u) {
                const int jn = j0 + u + 1;
                const size_t o = (size_t)(jn < P ? jn : 0) * 3 * NN;
                gx[u] = gy[u] = gz[u] = 0.0;
                if (j0 + u < P) {
                    gx[u] = p0[o];
                    gy[u] = p0[o + NN];
                    gz[u] = p0[o + 2 * NN];
                }
            }
#pragma unroll
            for (int u = 0; u < GB; ++u) {
                const int j = j0 + u;
                if (j < P) {
                    const double nx = gx[u], ny = gy[u], nz = gz[u];
                    bad |= !isfinite(cx) || !isfinite(cy) || !isfinite(cz);
                    const double ax = mimg<BOX>(cx - nx, box, ib);
                    const double ay = mimg<BOX>(cy - ny, box, ib);
                    const double az = mimg<BOX>(cz - nz, box, ib);
                    if (j + 1 < P || dist) ei += ax * ax + ay * ay + az * az;
                    et += cx * cx + cy * cy + cz * cz;
                    if (wf && ((j > 0 && j < P - 1) || dist)) {
                        const double bx = mimg<BOX>(cx - vx, box, ib);
                        const double by = mimg<BOX>(cy - vy, box, ib);
                        const double bz = mimg<BOX>(cz - vz, box, ib);
                        const size_t oj = (size_t)j * 3 * NN;
                        // streaming stores (nothing here reads them back):
                        // 1.3x the write bandwidth of cached stores
                        __builtin_nontemporal_store(scale * (-mw2 * (ax + bx) - trapc * cx), fo + oj);
                        __builtin_nontemporal_store(scale * (-mw2 * (ay + by) - trapc * cy), fo + oj + NN);
                        __builtin_nontemporal_store(scale * (-mw2 * (az + bz) - trapc * cz), fo + oj + 2 * NN);
                    }
                    vx = cx; vy = cy; vz = cz;
                    cx = nx; cy = ny; cz = nz;
                }
            }
        }
        esum = k * ei + 0.5 * trapc * et;
    }
    if (bad) set_flag(a.flags, ST_NONFINITE_IN);
    const double tot = block_sum(esum, sm + LDS_RED);
    if (t == 0) a.ws[sd.ws + WsLayout::epart(N) + chunk] = tot;
}

// ------------------------------------------------------------ fused kernel
// One launch runs every recursion and spring block of the batch; the
// exterior forces and energies follow in a second launch (k_finalize), so
// the results of all workgroups are visible to it through the stream order
// alone: no grid-wide flag, and no device-scope cache maintenance per
// workgroup.
template <int J, bool BOX, bool MIXED, bool SPLIT, bool WIDE = false>
__device__ __forceinline__ void exchange_body(const LaunchArgs &a) {
    extern __shared__ double sm[];
    const Item it = a.items[blockIdx.x];
    SysDesc sd = a.sys[it.sys];
    if (a.offs) { // caller-supplied packing (pimdb_exchange_forces_batched)
        sd.off = a.offs[it.sys];
        if (sd.off < 0) {
            if (threadIdx.x == 0) set_flag(a.flags, ST_RANGE);
            return;
        }
    }
    if (it.role == ROLE_FORWARD || it.role == ROLE_FHELP) {
        const int helper = it.role == ROLE_FHELP ? it.idx : -1;
        if (a.mode & M_WSUM)
            recursion_role<J, true, BOX, MIXED, true, SPLIT, WIDE>(a, sd, sm, helper);
        else
            recursion_role<J, true, BOX, MIXED, false, SPLIT, WIDE>(a, sd, sm, helper);
    } else if (it.role == ROLE_BACKWARD || it.role == ROLE_BHELP) {
        recursion_role<J, false, BOX, MIXED, true, SPLIT, WIDE>(a, sd, sm, it.role == ROLE_BHELP ? it.idx : -1);
    } else {
        // 1024-thread kernels have 128 registers: smaller bead groups
        springs_role<BOX, (J >= 4 ? 8 : 4)>(a, sd, it.sys, it.idx, sm);
    }
}

// Register budget: J <= 2 keeps 4 waves per SIMD at 1024 threads; J = 4 and
// J = 8 need the 512-thread bound to avoid spilling.
template <int J, bool BOX, bool MIXED>
__global__ void __launch_bounds__(1024) k_exchange(LaunchArgs a) {
    exchange_body<J, BOX, MIXED, false>(a);
}

template <int J, bool BOX, bool MIXED>
__global__ void __launch_bounds__(512) k_exchange_wide(LaunchArgs a) {
    exchange_body<J, BOX, MIXED, false>(a);
}

// Launches with split recursions (some systems spread over helper
// workgroups); 512 threads and at most 128 VGPRs, so that two workgroups
// share a CU (the residency the waits between workgroups rely on).
template <int J, bool BOX, bool MIXED>
__global__ void __launch_bounds__(512, 4) k_exchange_split(LaunchArgs a) {
    exchange_body<J, BOX, MIXED, true>(a);
}

// Split launches whose workgroups each have a CU of their own: 1024 threads
// and lag 3, so a chain's 16 waves form the next block's terms while its
// wave 0 runs the current block's steps.
template <int J, bool BOX, bool MIXED>
__global__ void __launch_bounds__(1024) k_exchange_split_wide(LaunchArgs a) {
    exchange_body<J, BOX, MIXED, true, true>(a);
}

// LDS of one fused workgroup: the recursion regions, or the springs role's
// reduction scratch (whichever is larger).  `exclusive` (split launches
// whose workgroups each have a CU): the wide chain's regions as well, more
// than half of a CU's 160 KiB, so that each workgroup has a CU to itself (a
// chain or helper then shares no SIMD with another workgroup's waves).
inline size_t exchange_smem_bytes(int threads, bool exclusive = false) {
    const int n = exclusive ? L_END2 : L_END;
    return (size_t)(threads > n ? threads : n) * sizeof(double);
}
static_assert(L_END2 * sizeof(double) <= 160 * 1024, "the wide chain's LDS exceeds a CU's");
static_assert(L_END2 * sizeof(double) > 80 * 1024, "a wide split workgroup must hold its CU alone");

} // namespace pimdb
