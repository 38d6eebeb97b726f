// HIP kernels for gfx950 other than the fused exchange launch (exchange.h):
// exterior-bead forces and energies (finalize), velocity-Verlet updates,
// status clearing, debug exports and the endpoint-spring table; and the
// dispatcher that picks the exchange launch variant.

#include "common.h"

namespace pimdb {

// ---------------------------------------------------------------- finalize
// One workgroup per system, after the recursions.  Exterior-bead forces
// (Theory, "Force on exterior beads") written in displacement form:
//   F_l^P = -m w^2 [ (r_l^P - r_l^{P-1}) + sum_{u<=l} Pr[l->u] (r_l^P - r_u^1)
//                    + Pr[l->l+1] (r_l^P - r_{l+1}^1) ]
//   F_l^1 = -m w^2 [ (r_l^1 - r_l^2) - sum_{l'>=l} Pr[l'->l] (r_l'^P - r_l^1)
//                    - Pr[l-1->l] (r_{l-1}^P - r_l^1) ]
// using that each row and each column of Pr sums to one.  The two Pr sums
// are rho * (weighted mean displacement) from the recursions.  Energy:
//   V^[1,N] = sum_l E_int(l) + sum_{l<N} s(l,l+1) + s(N,N) - ln(Z_f[N]) / beta.
template <bool BOX>
__device__ __forceinline__ void finalize(const LaunchArgs &a, const SysDesc sd, int si, double *red) {
    const int t = threadIdx.x, T = blockDim.x, N = sd.N, P = sd.P;
    const size_t NN = (size_t)N;
    const double *p0 = a.pos + sd.off;
    const double box = a.box, ib = a.inv_box;
    const bool dist = (a.mode & M_DIST) != 0;
    const bool wf = (a.mode & M_FORCES) && a.out && !dist;
    const bool we = (a.mode & M_ENERGY) && a.energy;
    if (!wf && !we) return;
    const double *wsb = a.ws + sd.ws;
    // the forward results live in the adjoint state when the forward half
    // wrote them there (M_SAVE) or the reverse half reads them (M_ADJOINT)
    const bool in_state = (a.mode & (M_ADJOINT | M_SAVE)) != 0;
    const double *fsrc = in_state ? a.state + sd.st : a.ws + sd.ws;
    const double *zfm = fsrc + (in_state ? StLayout::zf_m(N) : WsLayout::zf_m(N));
    const double *zfe = fsrc + (in_state ? StLayout::zf_e(N) : WsLayout::zf_e(N));
    const double *rf = fsrc + (in_state ? StLayout::rf(N) : WsLayout::rf(N));
    const double *zbm = wsb + WsLayout::zb_m(N);
    const double *zbe = wsb + WsLayout::zb_e(N);
    const double *rb = wsb + WsLayout::rb(N);
    const double scale = (a.mode & M_ADJOINT) ? -a.gscale[si] : 1.0;
    const double mw2 = sd.mw2;
    const double trapc = sd.m * a.trap_w2 / (double)P;
    const size_t oP = (size_t)(P - 1) * 3 * NN, oQ = (size_t)(P - 2) * 3 * NN, o2 = 3 * NN;
    double elink = 0.0;
    bool bad = false;
    // thread 0 starts the energy's interior-spring partials now, so their
    // round trip overlaps the particle loads (summed in chunk order below)
    constexpr int NEP = 8;
    double ep[NEP];
    const int nep = sd.nchunk < NEP ? sd.nchunk : NEP;
    if (we && t == 0) {
        for (int i = 0; i < NEP; ++i) ep[i] = wsb[WsLayout::epart(N) + (i < nep ? i : nep - 1)];
    }
    // Z_f[N], read once (also for the energy)
    const double zNm = dist ? 1.0 : zfm[N], zNe = dist ? 0.0 : zfe[N];
    if (!dist) {
        const double nInv = 1.0 / zNm;
        const int ne = (int)zNe;
        // Everything one particle q needs, read before any force is
        // written (the stores may alias the inputs as far as the compiler
        // knows, so a loop that reads and writes per particle waits a whole
        // memory round trip for each).
        struct In {
            double P[3], F[3], L[3], Q[3], B[3], K[3], rf[3], rb[3];
            double zf0m, zf0e, zb1m, zb1e, zf1m, zf1e, zb2m, zb2e;
        };
        auto load = [&](int q, In &x) {
            // link (or closing) spring of q: bead P of q to bead 1 of q+1 (q itself if last)
            const int r = q < N - 1 ? q + 1 : q;
            for (int c = 0; c < 3; ++c) {
                x.P[c] = p0[oP + c * NN + q];
                x.L[c] = p0[c * NN + r];
            }
            if (!wf) return;
            const int qm = q > 0 ? q - 1 : q; // bead P of q-1 (unused for q = 0)
            for (int c = 0; c < 3; ++c) {
                x.F[c] = p0[c * NN + q];
                x.Q[c] = p0[oQ + c * NN + q];
                x.B[c] = p0[o2 + c * NN + q];
                x.K[c] = p0[oP + c * NN + qm];
                x.rf[c] = rf[c * NN + q];
                x.rb[c] = rb[c * NN + q];
            }
            // Z_f[q+1] Z_b[q+2] (unused for the last particle; both in range)
            x.zf0m = zfm[q];
            x.zf0e = zfe[q];
            x.zb1m = zbm[q + 1];
            x.zb1e = zbe[q + 1];
            x.zf1m = zfm[q + 1];
            x.zf1e = zfe[q + 1];
            x.zb2m = zbm[q + 2];
            x.zb2e = zbe[q + 2];
        };
        auto emit = [&](int q, const In &x) {
            const double lx = mimg<BOX>(x.P[0] - x.L[0], box, ib);
            const double ly = mimg<BOX>(x.P[1] - x.L[1], box, ib);
            const double lz = mimg<BOX>(x.P[2] - x.L[2], box, ib);
            elink += lx * lx + ly * ly + lz * lz;
            if (!wf) return;
            // rho_l = Z_f[l] Z_b[l+1] / Z_f[N] for l = q+1 and l = q
            double rho, plink;
            if (q == N - 1) {
                rho = 1.0;
                plink = 0.0;
            } else {
                rho = ldexp(x.zf1m * x.zb2m * nInv, (int)x.zf1e + (int)x.zb2e - ne);
                plink = 1.0 - rho;
            }
            const double rhop = ldexp(x.zf0m * x.zb1m * nInv, (int)x.zf0e + (int)x.zb1e - ne);
            const double plinkp = q > 0 ? 1.0 - rhop : 0.0;
            const double Px = x.P[0], Py = x.P[1], Pz = x.P[2];
            const double Fx = x.F[0], Fy = x.F[1], Fz = x.F[2];
            // bead P
            const double ix = mimg<BOX>(Px - x.Q[0], box, ib);
            const double iy = mimg<BOX>(Py - x.Q[1], box, ib);
            const double iz = mimg<BOX>(Pz - x.Q[2], box, ib);
            double gx = ix + rho * x.rf[0] + plink * lx;
            double gy = iy + rho * x.rf[1] + plink * ly;
            double gz = iz + rho * x.rf[2] + plink * lz;
            const double fPx = scale * (-mw2 * gx - trapc * Px);
            const double fPy = scale * (-mw2 * gy - trapc * Py);
            const double fPz = scale * (-mw2 * gz - trapc * Pz);
            // bead 1
            const double jx = mimg<BOX>(Fx - x.B[0], box, ib);
            const double jy = mimg<BOX>(Fy - x.B[1], box, ib);
            const double jz = mimg<BOX>(Fz - x.B[2], box, ib);
            double hx = jx - rhop * x.rb[0], hy = jy - rhop * x.rb[1], hz = jz - rhop * x.rb[2];
            if (q > 0) {
                const double kx = mimg<BOX>(x.K[0] - Fx, box, ib);
                const double ky = mimg<BOX>(x.K[1] - Fy, box, ib);
                const double kz = mimg<BOX>(x.K[2] - Fz, box, ib);
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
        };
        // two particles per thread and pass, q and q + T (each thread still
        // meets its particles in the order t, t + T, t + 2T, ...)
        for (int q = t; q < N; q += 2 * T) {
            const bool two = q + T < N;
            In x0, x1;
            load(q, x0);
            load(two ? q + T : q, x1);
            emit(q, x0);
            if (two) emit(q + T, x1);
        }
    }
    if (we) {
        const double links = block_sum(elink, red);
        if (t == 0) {
            double E = 0.0;
            for (int i = 0; i < NEP; ++i)
                if (i < nep) E += ep[i];
            for (int c = NEP; c < sd.nchunk; ++c) E += wsb[WsLayout::epart(N) + c];
            if (!dist) E += sd.k * links - (log(zNm) + zNe * LN2) / sd.beta;
            bad |= !isfinite(E);
            a.energy[si] = E;
        }
    }
    if (bad) set_flag(a.flags, ST_NONFINITE_OUT);
}

// The split recursions' flags of one system (one workgroup).
__device__ __forceinline__ void clear_split_flags(const LaunchArgs &a, const SysDesc &sd) {
    if (sd.nhelp <= 0) return;
    const int nblk = (sd.N + 63) / 64;
    int *fl = (int *)(a.ws + sd.xs + XsLayout::flags(nblk));
    for (int64_t i = threadIdx.x; i < XsLayout::nflags(nblk); i += blockDim.x) fl[i] = 0;
}

__global__ void k_clear_flags(LaunchArgs a) { clear_split_flags(a, a.sys[blockIdx.x]); }

hipError_t launch_clear_flags(const LaunchArgs &a, int S, hipStream_t st) {
    if (S <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_clear_flags, dim3(S), dim3(256), 0, st, a);
    return hipGetLastError();
}

// One workgroup per system (memory-latency bound: 512 threads keep twice the
// loads of 256 in flight; at 1024 the 128-register limit makes it spill).
constexpr int FIN_T = 512;
template <bool BOX>
__global__ void __launch_bounds__(FIN_T) k_finalize(LaunchArgs a) {
    __shared__ double red[FIN_T];
    const int si = blockIdx.x;
    SysDesc sd = a.sys[si];
    clear_split_flags(a, sd); // the next evaluation starts with them at zero
    if (a.offs) {
        sd.off = a.offs[si];
        if (sd.off < 0) return; // flagged by the exchange launch
    }
    finalize<BOX>(a, sd, si, red);
}

hipError_t launch_finalize(const LaunchArgs &a, int S, hipStream_t st) {
    if (S <= 0) return hipSuccess;
    if (a.box > 0)
        hipLaunchKernelGGL(k_finalize<true>, dim3(S), dim3(FIN_T), 0, st, a);
    else
        hipLaunchKernelGGL(k_finalize<false>, dim3(S), dim3(FIN_T), 0, st, a);
    return hipGetLastError();
}

// ------------------------------------------------------ exchange dispatch
template <bool BOX, bool MIXED>
static int occupancy_j(int threads, int per_thread, int split) {
    switch (per_thread) {
    case 1: return exchange_variant_occupancy<1, BOX, MIXED>(threads, split);
    case 2: return exchange_variant_occupancy<2, BOX, MIXED>(threads, split);
    case 4: return exchange_variant_occupancy<4, BOX, MIXED>(threads, split);
    case 8: return exchange_variant_occupancy<8, BOX, MIXED>(threads, split);
    default: return 0;
    }
}

int exchange_occupancy(bool box, bool mixed, int threads, int per_thread, int split) {
    if (box) return mixed ? occupancy_j<true, true>(threads, per_thread, split)
                          : occupancy_j<true, false>(threads, per_thread, split);
    return mixed ? occupancy_j<false, true>(threads, per_thread, split)
                 : occupancy_j<false, false>(threads, per_thread, split);
}

template <bool BOX, bool MIXED>
static hipError_t launch_j(const LaunchArgs &a, int nitems, int threads, int per_thread, int split, hipStream_t st) {
    switch (per_thread) {
    case 1: return launch_exchange_variant<1, BOX, MIXED>(a, nitems, threads, split, st);
    case 2: return launch_exchange_variant<2, BOX, MIXED>(a, nitems, threads, split, st);
    case 4: return launch_exchange_variant<4, BOX, MIXED>(a, nitems, threads, split, st);
    case 8: return launch_exchange_variant<8, BOX, MIXED>(a, nitems, threads, split, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_exchange(const LaunchArgs &a, int nitems, int threads, int per_thread, int split, hipStream_t st) {
    if (nitems <= 0) return hipSuccess;
    // the periodic variants with box 0 form every pair displacement directly
    // (the minimum image of d with L = 0 is d exactly): the open FP64 path
    // without the dot-product expansion
    const bool box = a.box > 0 || a.direct;
    if (box) return a.mixed ? launch_j<true, true>(a, nitems, threads, per_thread, split, st)
                            : launch_j<true, false>(a, nitems, threads, per_thread, split, st);
    return a.mixed ? launch_j<false, true>(a, nitems, threads, per_thread, split, st)
                   : launch_j<false, false>(a, nitems, threads, per_thread, split, st);
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
        exp2x(fmax(fma(sd.kappa, q2(l, u), -sd.kappa * q2(l, r)), XLO), p, nr);
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
        // rows start at arbitrary offsets, so a row segment covers partial
        // cache lines at its ends: streaming stores measured faster for the
        // 4-byte table (2.0 vs 1.8 TB/s at N=4096) and slower for the 8-byte
        // one (2.8 vs 4.0 TB/s), which keeps cached stores
        if (F32)
            __builtin_nontemporal_store((float)(k * sqlen<true>(dx, dy, dz)), (float *)dst + o);
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
