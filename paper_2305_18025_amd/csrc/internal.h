// Internal types shared by the host API (api.cpp) and the kernels
// (kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pimdb {

// Roles of a workgroup in the fused evaluation launch.
enum Role : int32_t {
    ROLE_FORWARD = 0,  // forward recursion of one system (its serial chain only, when split)
    ROLE_BACKWARD = 1, // backward recursion of one system (its serial chain only, when split)
    ROLE_SPRINGS = 2,  // interior springs of one block of particles
    ROLE_FHELP = 3,    // helper of a split forward recursion: accumulators of some blocks
    ROLE_BHELP = 4,    // helper of a split backward recursion
};

// Evaluation modes (bit set).
enum ModeBits : int32_t {
    M_FWD = 1,        // run forward recursions
    M_BWD = 2,        // run backward recursions
    M_WSUM = 4,       // forward recursion accumulates weighted displacements
    M_FORCES = 8,     // write forces (interior by springs, exterior by finalize)
    M_ENERGY = 16,    // write energies
    M_ADJOINT = 32,   // forces scaled by -grad_energy[s]; forward results read from state
    M_SAVE = 64,      // forward results written to state instead of the workspace
    M_DIST = 128,     // distinguishable particles: springs close each ring, no recursions
};

// Per-system descriptor (device table, built by pimdb_set_batch).
struct SysDesc {
    int64_t off;    // element offset of the system in packed (P,3,N) arrays
    int64_t ws;     // offset in doubles of the system's region in the workspace
    int64_t st;     // offset in doubles of the system's region in the adjoint state
    int64_t xs;     // offset in doubles of the split recursions' exchange area (nhelp > 0)
    int32_t N, P;
    int32_t nchunk; // number of ROLE_SPRINGS items (ceil(N / threads))
    int32_t nhelp;  // helper workgroups per recursion direction (0: one workgroup per recursion)
    double beta, m, omegaP;
    double k;       // (1/2) m omega_P^2
    double mw2;     // m omega_P^2
    double kappa;   // -beta k log2(e): spring exponent factor in log2 units
};

// One workgroup's job.
struct Item {
    int32_t sys;
    int32_t role;
    int32_t idx; // chunk index for ROLE_SPRINGS
    int32_t pad;
};

// Per-system workspace layout, offsets in doubles from SysDesc::ws.
//   zf_m[N+1], zf_e[N+1] : forward  Z_f[v] = zf_m * 2^zf_e, v = 0..N
//   zb_m[N+2], zb_e[N+2] : backward Z_b[u] = zb_m * 2^zb_e, u = 1..N+1
//   rf[3][N]             : forward-weighted mean endpoint displacement
//   rb[3][N]             : backward-weighted mean endpoint displacement
//   epart[nchunk]        : interior/trap energy partial sums
//   cpre[N+1]            : gauge prefix sums (debug exports only)
struct WsLayout {
    static __host__ __device__ inline int64_t zf_m(int N) { return 0; }
    static __host__ __device__ inline int64_t zf_e(int N) { return (int64_t)N + 1; }
    static __host__ __device__ inline int64_t zb_m(int N) { return 2 * ((int64_t)N + 1); }
    static __host__ __device__ inline int64_t zb_e(int N) { return 2 * ((int64_t)N + 1) + (N + 2); }
    static __host__ __device__ inline int64_t rf(int N) { return 2 * ((int64_t)N + 1) + 2 * ((int64_t)N + 2); }
    static __host__ __device__ inline int64_t rb(int N) { return rf(N) + 3 * (int64_t)N; }
    static __host__ __device__ inline int64_t epart(int N) { return rb(N) + 3 * (int64_t)N; }
    static __host__ __device__ inline int64_t cpre(int N, int nchunk) { return epart(N) + nchunk; }
    static __host__ __device__ inline int64_t total(int N, int nchunk) { return cpre(N, nchunk) + N + 1; }
};

// Exchange area of a split recursion, offsets in doubles from SysDesc::xs
// (nblk = ceil(N / 64) blocks; direction d = 0 forward, 1 backward):
//   pub_zl[nblk][64]  step values the chain publishes (what the panels use)
//   pub_ze[nblk][64]  their exponents (ints)
//   del_acc[nblk][4][64]  accumulators {A, Wx, Wy, Wz} helpers deliver
//   del_e[nblk][64]   their exponents (ints)
// then, for both directions, the flags (ints): [d][0][nblk] block published,
// [d][1][nblk] accumulator delivered; zero between evaluations (cleared by
// the finalize launch).
struct XsLayout {
    static __host__ __device__ inline int64_t dir(int nblk) { return (int64_t)nblk * 384; }
    static __host__ __device__ inline int64_t pub_zl(int nblk, int d) { return d * dir(nblk); }
    static __host__ __device__ inline int64_t pub_ze(int nblk, int d) { return pub_zl(nblk, d) + 64 * (int64_t)nblk; }
    static __host__ __device__ inline int64_t del_acc(int nblk, int d) { return pub_ze(nblk, d) + 32 * (int64_t)nblk; }
    static __host__ __device__ inline int64_t del_e(int nblk, int d) { return del_acc(nblk, d) + 256 * (int64_t)nblk; }
    static __host__ __device__ inline int64_t flags(int nblk) { return 2 * dir(nblk); }
    static __host__ __device__ inline int64_t nflags(int nblk) { return 4 * (int64_t)nblk; } // ints
    static __host__ __device__ inline int64_t total(int nblk) { return 2 * dir(nblk) + 2 * (int64_t)nblk; }
};

// Adjoint state layout per system, offsets in doubles from SysDesc::st:
//   zf_m[N+1], zf_e[N+1], rf[3][N]
struct StLayout {
    static __host__ __device__ inline int64_t zf_m(int N) { return 0; }
    static __host__ __device__ inline int64_t zf_e(int N) { return (int64_t)N + 1; }
    static __host__ __device__ inline int64_t rf(int N) { return 2 * ((int64_t)N + 1); }
    static __host__ __device__ inline int64_t total(int N) { return 2 * ((int64_t)N + 1) + 3 * (int64_t)N; }
};

// Workspace header (bytes): the status word.
constexpr int64_t WS_HEADER_BYTES = 256;

struct LaunchArgs {
    const SysDesc *sys;
    const Item *items;
    const double *pos;
    double *out;           // forces / gradient (may be null: no force writes)
    double *energy;        // per-system energies (may be null)
    double *ws;            // workspace doubles (after the header)
    int32_t *flags;        // status word
    double *state;         // adjoint state (M_SAVE writes it, M_ADJOINT reads it)
    const double *gscale;  // adjoint: grad of energy per system
    const int64_t *offs;   // caller's element offset per system (device array), or null: SysDesc::off
    double box, inv_box;   // periodic box (0 = open)
    double trap_w2;        // trap omega^2 (0 = none)
    int32_t mode;
    int32_t mixed;         // 1: FP32 compensated endpoint spring lengths
    int32_t direct;        // 1: direct-form pair lengths for open boundaries (host-side choice of variant)
    int32_t help_rows;     // split recursions: row waves per helper workgroup
    uint64_t wait_ticks;   // time limit of a split recursion's wait, 100 MHz clock ticks
};

// Kernel launch entry points (kernels.hip).  launch_exchange picks one of
// the variants compiled from exchange_inst.hip (J accumulator rows per
// thread, periodic box, mixed precision).
// `split`: 0 whole recursions; 1 the variant with split recursions (J = 1,
// 2; 512 threads); 2 the same with one workgroup per CU (more LDS than
// half a CU's).
template <int J, bool BOX, bool MIXED>
hipError_t launch_exchange_variant(const LaunchArgs &a, int nitems, int threads, int split, hipStream_t st);
hipError_t launch_exchange(const LaunchArgs &a, int nitems, int threads, int per_thread, int split, hipStream_t st);
// Workgroups of one exchange variant resident per CU at this width (the
// occupancy the split recursions' waits rely on).
template <int J, bool BOX, bool MIXED>
int exchange_variant_occupancy(int threads, int split);
int exchange_occupancy(bool box, bool mixed, int threads, int per_thread, int split);
hipError_t launch_finalize(const LaunchArgs &a, int S, hipStream_t st);
hipError_t launch_clear(int32_t *p, int64_t n, hipStream_t st);
// Zero the split recursions' flags of every split system of the batch.
hipError_t launch_clear_flags(const LaunchArgs &a, int S, hipStream_t st);
// Element range of one system handled by one workgroup of the MD kernels.
struct EChunk {
    int32_t sys;
    int32_t pad;
    int64_t begin, end; // element range in packed arrays
};

// Workspace of the original (cubic) algorithm for one system of N
// particles with P beads, offsets in doubles from the system's region; NB =
// 3 P N right-hand sides (bead derivatives), b = ((l-1) P + j-1) 3 + c:
//   ein[N]        interior spring sums of each particle (without k)
//   lnk[N]        link spring of particle l to l+1 (without k; 0 for l = N)
//   V[N+1]        V^[1,v], v = 0..N
//   Et[N][N]      [v-1][u-1] = E^[u,v] for u <= v, 0 above
//   Er[N][N]      [u-1][v-1] = E^[u,v] (the transpose)
//   W[N][N]       [g][v-1] = weight of cycle [g+1, v] in V^[1,v] (g < v), 0 else
//   C[N+1][N]     [L][v-1] = sum_{g < L} W[g][v-1]
//   T[N][3]       last-bead derivative sums at v = l
//   G[NB/256][N][256]  [b/256][v-1][b%256] = dV^[1,v] / dx_b, stored for v >= l(b)
//                 (the 256 right-hand sides of a workgroup contiguous per v:
//                 its history is one contiguous region)
struct OrigLayout {
    static __host__ __device__ inline int64_t ein(int64_t N) { return 0; }
    static __host__ __device__ inline int64_t lnk(int64_t N) { return N; }
    static __host__ __device__ inline int64_t V(int64_t N) { return 2 * N; }
    static __host__ __device__ inline int64_t Et(int64_t N) { return 3 * N + 1; }
    static __host__ __device__ inline int64_t Er(int64_t N) { return Et(N) + N * N; }
    static __host__ __device__ inline int64_t W(int64_t N) { return Er(N) + N * N; }
    static __host__ __device__ inline int64_t C(int64_t N) { return W(N) + N * N; }
    static __host__ __device__ inline int64_t T(int64_t N) { return C(N) + (N + 1) * N; }
    static __host__ __device__ inline int64_t G(int64_t N) { return (T(N) + 3 * N + 31) / 32 * 32; }
    static __host__ __device__ inline int64_t G_rhs(int64_t N, int64_t P) { return (3 * P * N + 255) / 256 * 256; }
    static __host__ __device__ inline int64_t total(int64_t N, int64_t P) { return G(N) + N * G_rhs(N, P); }
};

// One system's evaluation by the original algorithm.
struct OrigArgs {
    const double *pos;  // the system's (P,3,N) positions
    double *out;        // its forces (null: energy only)
    double *energy;     // its energy (may be null)
    double *ws;         // its OrigLayout region
    int32_t *flags;     // status word
    int32_t N, P;
    double beta, k, mw2;
    double box, inv_box;
    double trapc;       // trap force coefficient m w^2 / P (0 = none)
    int32_t two_term;   // 1: the two-candidate shift of the forward recurrence
    int32_t pad;
};
hipError_t launch_original(const OrigArgs &a, hipStream_t st);

// Scaled pair interaction: one workgroup per item, bead slice j of system
// sys, particles i0 .. i0 + iblock - 1 against every particle of the slice.
struct PairItem {
    int32_t sys, j, i0, pad;
};
struct PairArgs {
    const SysDesc *sys;
    const PairItem *items;
    const int32_t *beg;    // first item of each system (S + 1 entries)
    const int64_t *offs;   // caller's element offset per system, or null: SysDesc::off
    const double *pos;
    double *out;           // forces (or the gradient), may be null
    double *energy;        // per-system energies, may be null
    double *epart;         // one energy partial per item (workspace)
    const double *gscale;  // gradient mode: per-system factor (null: 1)
    int32_t *flags;        // status word
    double box, inv_box;
    double c2;             // -log2(e) / (2 sigma^2): exponent of U in log2 units per r^2
    double g, inv_s2;      // U(0) and 1 / sigma^2
    int32_t sign;          // +1: forces -dU/dr; -1: the gradient (adjoint)
    int32_t accumulate;    // 1: add to out and energy; 0: overwrite them
    int32_t iblock;        // particles per item (the workgroup size)
    int32_t pad;
};
hipError_t launch_pair(const PairArgs &a, int nitems, int S, hipStream_t st);

hipError_t launch_md_update(const SysDesc *sys, const EChunk *chunks, int nchunks, double *pos,
                            double *vel, const double *forces, double dt, int drift, hipStream_t st);
hipError_t launch_debug_prefix(const LaunchArgs &a, int s, int threads, hipStream_t st);
hipError_t launch_debug_table(const LaunchArgs &a, int s, int N, int what, double *dst, hipStream_t st);
hipError_t launch_endpoint_springs(const LaunchArgs &a, int s, int N, int as_float, void *dst, hipStream_t st);

} // namespace pimdb
