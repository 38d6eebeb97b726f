/*
 * Oracle body: plain, slow, literal CPU implementation of the bosonic
 * exchange potential V^[1,N] and its bead forces.  TEST INFRASTRUCTURE ONLY.
 *
 * This file is included twice by pimdb_oracle.c, once with REAL = double
 * (suffix _f64) and once with REAL = long double (x87 80-bit, suffix _f80).
 * The arithmetic is identical; only the working precision differs.  The
 * long-double build is the high-precision reference used to attribute the
 * rounding error of any FP64 result.
 *
 * Notation (paper, Sec. "Background: cubic scaling bosonic PIMD"):
 *   N particles, P beads, bead positions r_l^j, l = 1..N, j = 1..P, d = 3.
 *   k = (1/2) m omega_P^2 is the spring prefactor; m omega_P^2 = 2k.
 * Positions arrive as R[(l*P + j)*3 + c] with 0-based l, j, c (row-major
 * N x P x 3), i.e. particle-major; this is the oracle's own layout.
 *
 * Periodic boxes: when L > 0 every spring displacement is replaced by its
 * minimum image d - L*rint(d/L) (round half to even), applied per spring.
 * The paper only states that periodic boundary conditions were used; this
 * per-spring reading keeps every formula below unchanged.
 */

#define CAT_(a, b) a##b
#define CAT(a, b) CAT_(a, b)
#define FN(name) CAT(name, SFX)

/* minimum-image displacement of one component */
static REAL FN(mi_)(REAL d, REAL L) {
    if (L > 0) return d - L * RINT(d / L);
    return d;
}

/* squared distance |r_a^ja - r_b^jb|^2 (0-based indices), minimum image */
static REAL FN(dist2_)(const double *R, int P, int a, int ja, int b, int jb, REAL L) {
    REAL s = 0;
    for (int c = 0; c < 3; ++c) {
        REAL d = FN(mi_)((REAL)R[((size_t)a * P + ja) * 3 + c] - (REAL)R[((size_t)b * P + jb) * 3 + c], L);
        s += d * d;
    }
    return s;
}

/* displacement vector r_a^ja - r_b^jb (minimum image) */
static void FN(disp_)(const double *R, int P, int a, int ja, int b, int jb, REAL L, REAL out[3]) {
    for (int c = 0; c < 3; ++c)
        out[c] = FN(mi_)((REAL)R[((size_t)a * P + ja) * 3 + c] - (REAL)R[((size_t)b * P + jb) * 3 + c], L);
}

/*
 * The quadratic-scaling potential and forces ("Fast PIMD-B"), computed from
 * the defining equations of the paper's main text:
 *   - interior spring energy E_int(l): the P-1 springs j -> j+1 of particle
 *     l that no permutation changes (Theory, "Reducing the potential",
 *     definition of the interior energy);
 *   - cycle energy E^[u,v]: the energy of the ring through particles u..v,
 *     i.e. the interior springs of each of them, the link from bead P of l
 *     to bead 1 of l+1 for l = u..v-1, and the spring closing the ring from
 *     bead P of v to bead 1 of u (Background, definition of the cycle
 *     energies).  For each u the open part is summed particle by particle
 *     as v grows and the closing spring is added on top;
 *   - V^[1,v] from the recurrence over the length of the cycle that contains
 *     v (Background, the recurrence defining the potential), V^[1,0] = 0;
 *   - V^[u,N] from the backward recursion with weight 1/l on the last
 *     particle l of the cycle that starts at u (Theory, "Connection
 *     probabilities"), V^[N+1,N] = 0;
 *   - every exponential sum is evaluated with a shift that is exact in exact
 *     arithmetic (appendix "Numerical Stability"): shift_mode 0 takes the
 *     smallest exponent of the sum (largest term 1), shift_mode 1 the two
 *     candidates the paper uses for small trapped systems;
 *   - Pr[l -> l+1] as the complement of the probability that l and l+1 lie
 *     in different cycles (Theory, direct-link expression), Pr[l -> l'] for
 *     l' <= l from the cycle-closing expression (Methods, "Expressions for
 *     connection probabilities"), and 0 for l' > l+1 (Methods: a particle
 *     links forward only to the next label);
 *   - forces on interior beads from the ordinary ring-polymer expression
 *     (Theory, "Force on interior beads"), and on beads 1 and P as the
 *     probability-weighted sums over every possible neighbour l' = 1..N
 *     (Theory, "Force on exterior beads").
 *
 * Outputs (all optional except V): V = V^[1,N]; F = -grad V in the
 * oracle layout; Vf[0..N] = V^[1,v]; Vb[0..N+1] with Vb[u] = V^[u,N] for
 * u = 1..N+1 (Vb[0] unused, set to 0); Pr[(l-1)*N + (l'-1)] = Pr[l -> l'];
 * E[(u-1)*N + (v-1)] = E^[u,v] for u <= v (0 elsewhere); Eint[l-1].
 * Returns 0, or -1 on invalid arguments, -2 on allocation failure.
 */

/* -(1/beta) ln( sum_i w_i exp(-beta x_i) ) for n exponents x and weights w,
 * with the exponents shifted by sh before exponentiating. */
static REAL FN(neg_log_sum_)(int n, const REAL *x, const REAL *w, REAL beta, REAL sh) {
    REAL acc = 0;
    for (int i = 0; i < n; ++i) acc += w[i] * EXP(-beta * (x[i] - sh));
    return sh - LOG(acc) / beta;
}

static REAL FN(min_of_)(int n, const REAL *x) {
    REAL s = x[0];
    for (int i = 1; i < n; ++i)
        if (x[i] < s) s = x[i];
    return s;
}

int FN(orc_alg1)(int N, int P, const double *R, double beta, double m, double omegaP, double L,
                 int shift_mode, double *V_out, double *F_out, double *Vf_out, double *Vb_out,
                 double *Pr_out, double *E_out, double *Eint_out) {
    if (N < 1 || P < 2 || !(beta > 0) || !(m > 0) || !(omegaP > 0) || !(L >= 0) || !R || !V_out)
        return -1;
    const REAL b = (REAL)beta;
    const REAL Lr = (REAL)L;
    const REAL k = (REAL)0.5 * (REAL)m * (REAL)omegaP * (REAL)omegaP; /* spring prefactor */
    const REAL mw2 = (REAL)m * (REAL)omegaP * (REAL)omegaP;

    REAL *Eint = (REAL *)calloc((size_t)N + 2, sizeof(REAL));          /* 1-based */
    REAL *E = (REAL *)calloc((size_t)(N + 2) * (N + 2), sizeof(REAL)); /* E[u*(N+2)+v] */
    REAL *Vf = (REAL *)calloc((size_t)N + 2, sizeof(REAL));
    REAL *Vb = (REAL *)calloc((size_t)N + 2, sizeof(REAL));
    REAL *Pr = (REAL *)calloc((size_t)(N + 2) * (N + 2), sizeof(REAL)); /* Pr[l*(N+2)+l'] */
    REAL *x = (REAL *)calloc((size_t)N + 2, sizeof(REAL));
    REAL *w = (REAL *)calloc((size_t)N + 2, sizeof(REAL));
    if (!Eint || !E || !Vf || !Vb || !Pr || !x || !w) {
        free(Eint); free(E); free(Vf); free(Vb); free(Pr); free(x); free(w);
        return -2;
    }
#define EE(u, v) E[(size_t)(u) * (N + 2) + (v)]
#define PR(l, lp) Pr[(size_t)(l) * (N + 2) + (lp)]
    /* squared length of the spring between bead ja of particle a and bead jb
     * of particle bb (1-based), minimum image when periodic */
#define S2(a, ja, bb, jb) FN(dist2_)(R, P, (a) - 1, (ja) - 1, (bb) - 1, (jb) - 1, Lr)

    /* interior spring energies */
    for (int l = 1; l <= N; ++l) {
        REAL s = 0;
        for (int j = 1; j <= P - 1; ++j) s += S2(l, j, l, j + 1);
        Eint[l] = k * s;
    }
    /* cycle energies: ring through u..v = open chain u..v + closing spring */
    for (int u = 1; u <= N; ++u) {
        REAL open = 0; /* interior springs of u..v and the links u -> u+1 .. v-1 -> v */
        for (int v = u; v <= N; ++v) {
            if (v > u) open += k * S2(v - 1, P, v, 1);
            open += Eint[v];
            EE(u, v) = open + k * S2(v, P, u, 1);
        }
    }
    /* forward potentials: exp(-b V^[1,v]) = (1/v) sum_{u=1}^{v} exp(-b(V^[1,u-1] + E^[u,v])) */
    Vf[0] = 0;
    for (int v = 1; v <= N; ++v) {
        for (int u = 1; u <= v; ++u) {
            x[u - 1] = Vf[u - 1] + EE(u, v);
            w[u - 1] = (REAL)1 / (REAL)v;
        }
        REAL sh;
        if (shift_mode == 1) { /* the two candidates: whole ring 1..v, or v alone after V^[1,v-1] */
            sh = x[0];
            if (x[v - 1] < sh) sh = x[v - 1];
        } else {
            sh = FN(min_of_)(v, x);
        }
        Vf[v] = FN(neg_log_sum_)(v, x, w, b, sh);
    }
    /* backward potentials: exp(-b V^[u,N]) = sum_{l=u}^{N} (1/l) exp(-b(E^[u,l] + V^[l+1,N])) */
    Vb[N + 1] = 0;
    for (int u = N; u >= 1; --u) {
        const int n = N - u + 1;
        for (int l = u; l <= N; ++l) {
            x[l - u] = EE(u, l) + Vb[l + 1];
            w[l - u] = (REAL)1 / (REAL)l;
        }
        REAL sh;
        if (shift_mode == 1) { /* u alone before V^[u+1,N], or the whole ring u..N */
            sh = x[0];
            if (x[n - 1] < sh) sh = x[n - 1];
        } else {
            sh = FN(min_of_)(n, x);
        }
        Vb[u] = FN(neg_log_sum_)(n, x, w, b, sh);
    }
    const REAL VN = Vf[N];
    /* connection probabilities Pr[l -> l'] for every pair */
    for (int l = 1; l <= N; ++l) {
        for (int lp = 1; lp <= N; ++lp) {
            REAL p = 0;
            if (lp == l + 1) /* 1 - exp(-b(V^[1,l] + V^[l+1,N] - V^[1,N])), as -expm1 */
                p = -EXPM1(-b * (Vf[l] + Vb[l + 1] - VN));
            else if (lp <= l) /* the ring lp..l closes: (1/l) exp(-b(V^[1,lp-1] + E^[lp,l] + V^[l+1,N] - V^[1,N])) */
                p = EXP(-b * (Vf[lp - 1] + EE(lp, l) + Vb[l + 1] - VN)) / (REAL)l;
            PR(l, lp) = p;
        }
    }

    if (F_out) {
        for (int l = 1; l <= N; ++l) {
            /* interior beads: -m w^2 (2 r^j - r^{j+1} - r^{j-1}) */
            for (int j = 2; j <= P - 1; ++j) {
                REAL up[3], dn[3];
                FN(disp_)(R, P, l - 1, j - 1, l - 1, j, Lr, up);     /* r^j - r^{j+1} */
                FN(disp_)(R, P, l - 1, j - 1, l - 1, j - 2, Lr, dn); /* r^j - r^{j-1} */
                for (int c = 0; c < 3; ++c)
                    F_out[(((size_t)l - 1) * P + (j - 1)) * 3 + c] = (double)(-mw2 * (up[c] + dn[c]));
            }
            /* bead 1: its predecessor is bead P of l' with probability Pr[l' -> l];
             * bead P: its successor is bead 1 of l' with probability Pr[l -> l'] */
            REAL f1[3] = {0, 0, 0}, fP[3] = {0, 0, 0};
            REAL in1[3], inP[3];
            FN(disp_)(R, P, l - 1, 0, l - 1, 1, Lr, in1);     /* r_l^1 - r_l^2 */
            FN(disp_)(R, P, l - 1, P - 1, l - 1, P - 2, Lr, inP); /* r_l^P - r_l^{P-1} */
            for (int lp = 1; lp <= N; ++lp) {
                REAL d[3];
                const REAL pin = PR(lp, l), pout = PR(l, lp);
                FN(disp_)(R, P, l - 1, 0, lp - 1, P - 1, Lr, d); /* r_l^1 - r_l'^P */
                for (int c = 0; c < 3; ++c) f1[c] -= pin * mw2 * (in1[c] + d[c]);
                FN(disp_)(R, P, l - 1, P - 1, lp - 1, 0, Lr, d); /* r_l^P - r_l'^1 */
                for (int c = 0; c < 3; ++c) fP[c] -= pout * mw2 * (inP[c] + d[c]);
            }
            for (int c = 0; c < 3; ++c) {
                F_out[(((size_t)l - 1) * P + 0) * 3 + c] = (double)f1[c];
                F_out[(((size_t)l - 1) * P + (P - 1)) * 3 + c] = (double)fP[c];
            }
        }
    }
    *V_out = (double)VN;
    if (Vf_out)
        for (int v = 0; v <= N; ++v) Vf_out[v] = (double)Vf[v];
    if (Vb_out) {
        Vb_out[0] = 0;
        for (int u = 1; u <= N + 1; ++u) Vb_out[u] = (double)Vb[u];
    }
    if (Pr_out)
        for (int l = 1; l <= N; ++l)
            for (int lp = 1; lp <= N; ++lp) Pr_out[(size_t)(l - 1) * N + (lp - 1)] = (double)PR(l, lp);
    if (E_out)
        for (int u = 1; u <= N; ++u)
            for (int v = 1; v <= N; ++v) E_out[(size_t)(u - 1) * N + (v - 1)] = u <= v ? (double)EE(u, v) : 0.0;
    if (Eint_out)
        for (int l = 1; l <= N; ++l) Eint_out[l - 1] = (double)Eint[l];
#undef EE
#undef PR
#undef S2
    free(Eint); free(E); free(Vf); free(Vb); free(Pr); free(x); free(w);
    return 0;
}

/*
 * Original PIMD-B (Alg. 2 of the appendix), the cubic algorithm that the
 * paper states produces exactly the same potential and forces:
 *   - each cycle energy E^[u,v] directly from its definition (Background,
 *     definition of the cycle energy as a double sum; the sums run over the
 *     particles u..v of the cycle), O(P(v-u+1)) each;
 *   - the same forward recurrence for V^[1,v] (full max shift);
 *   - forces from the derivative of that recurrence, evaluated separately
 *     for every bead:  grad V^[1,v] = sum_k w_k (grad E^[v-k+1,v] +
 *     grad V^[1,v-k]) with w_k = exp(-beta(V^[1,v-k] + E^[v-k+1,v] -
 *     V^[1,v])) / v, which is what differentiating the recurrence gives
 *     (the printed exponent is garbled; this is the derivative).
 *   The bead derivative of a cycle energy uses the ring neighbours inside
 *   the cycle: r_l^0 = r_{l-1}^P and r_l^{P+1} = r_{l+1}^1, except that the
 *   cycle closes with r_u^0 = r_v^P and r_v^{P+1} = r_u^1.
 * O(P N^3) time.  Returns 0 or -1 / -2 as orc_alg1.
 */
int FN(orc_alg2)(int N, int P, const double *R, double beta, double m, double omegaP, double L,
                 double *V_out, double *F_out) {
    if (N < 1 || P < 2 || !(beta > 0) || !(m > 0) || !(omegaP > 0) || !(L >= 0) || !R || !V_out)
        return -1;
    const REAL b = (REAL)beta;
    const REAL Lr = (REAL)L;
    const REAL k = (REAL)0.5 * (REAL)m * (REAL)omegaP * (REAL)omegaP;
    const REAL mw2 = (REAL)m * (REAL)omegaP * (REAL)omegaP;
    REAL *E = (REAL *)calloc((size_t)(N + 1) * (N + 1), sizeof(REAL));
    REAL *Vf = (REAL *)calloc((size_t)N + 1, sizeof(REAL));
    REAL *W = (REAL *)calloc((size_t)(N + 1) * (N + 1), sizeof(REAL)); /* W[u*(N+1)+v] weight of cycle [u,v] in V^[1,v] */
    REAL *G = (REAL *)calloc((size_t)N + 1, sizeof(REAL));
    if (!E || !Vf || !W || !G) {
        free(E); free(Vf); free(W); free(G);
        return -2;
    }
#define EE(u, v) E[(size_t)(u) * (N + 1) + (v)]
#define WW(u, v) W[(size_t)(u) * (N + 1) + (v)]
#define S2(a, ja, bb, jb) FN(dist2_)(R, P, (a) - 1, (ja) - 1, (bb) - 1, (jb) - 1, Lr)
    for (int v = 1; v <= N; ++v) {
        for (int u = 1; u <= v; ++u) {
            REAL s = 0;
            for (int l = u; l <= v; ++l)
                for (int j = 1; j <= P - 1; ++j) s += S2(l, j + 1, l, j);
            for (int l = u; l <= v - 1; ++l) s += S2(l + 1, 1, l, P);
            s += S2(u, 1, v, P);
            EE(u, v) = k * s;
        }
    }
    Vf[0] = 0;
    for (int v = 1; v <= N; ++v) {
        REAL sh = Vf[0] + EE(1, v);
        for (int u = 2; u <= v; ++u)
            if (Vf[u - 1] + EE(u, v) < sh) sh = Vf[u - 1] + EE(u, v);
        REAL acc = 0;
        for (int u = 1; u <= v; ++u) acc += EXP(-b * (Vf[u - 1] + EE(u, v) - sh));
        Vf[v] = sh - LOG(acc / (REAL)v) / b;
        for (int u = 1; u <= v; ++u) WW(u, v) = EXP(-b * (Vf[u - 1] + EE(u, v) - Vf[v])) / (REAL)v;
    }
    if (F_out) {
        /* derivative of E^[u,v] with respect to bead (l, j), component c */
        for (int l = 1; l <= N; ++l) {
            for (int j = 1; j <= P; ++j) {
                for (int c = 0; c < 3; ++c) {
                    G[0] = 0;
                    for (int v = 1; v <= N; ++v) {
                        REAL g = 0;
                        for (int u = 1; u <= v; ++u) {
                            REAL dE = 0;
                            if (u <= l && l <= v) {
                                /* previous bead of (l, j) inside cycle [u, v] */
                                int pa, pj, na, nj;
                                if (j > 1) { pa = l; pj = j - 1; }
                                else if (l > u) { pa = l - 1; pj = P; }
                                else { pa = v; pj = P; }
                                if (j < P) { na = l; nj = j + 1; }
                                else if (l < v) { na = l + 1; nj = 1; }
                                else { na = u; nj = 1; }
                                REAL d1[3], d2[3];
                                FN(disp_)(R, P, l - 1, j - 1, pa - 1, pj - 1, Lr, d1);
                                FN(disp_)(R, P, l - 1, j - 1, na - 1, nj - 1, Lr, d2);
                                dE = mw2 * (d1[c] + d2[c]);
                            }
                            g += WW(u, v) * (dE + G[u - 1]);
                        }
                        G[v] = g;
                    }
                    F_out[(((size_t)l - 1) * P + (j - 1)) * 3 + c] = (double)(-G[N]);
                }
            }
        }
    }
    *V_out = (double)Vf[N];
#undef EE
#undef WW
#undef S2
    free(E); free(Vf); free(W); free(G);
    return 0;
}

/*
 * V^[u,N] from its definition in the appendix ("Connection Probabilities",
 * definition of the backward potentials): for fixed u, the recursion over
 * the upper index M = u..N,
 *     exp(-beta V^[u,M]) = (1/M) sum_{k=1}^{M-u+1} exp(-beta(V^[u,M-k] + E^[M-k+1,M])),
 * with V^[u,u-1] = 0.  Cycle energies come from their definition (direct
 * double sum), not from the incremental recurrence.  O(P N^3 + N^3).
 * Vb_out[u] for u = 1..N (Vb_out[0] set to 0).
 */
int FN(orc_backward_def)(int N, int P, const double *R, double beta, double m, double omegaP, double L,
                         double *Vb_out) {
    if (N < 1 || P < 2 || !(beta > 0) || !(m > 0) || !(omegaP > 0) || !(L >= 0) || !R || !Vb_out)
        return -1;
    const REAL b = (REAL)beta;
    const REAL Lr = (REAL)L;
    const REAL k = (REAL)0.5 * (REAL)m * (REAL)omegaP * (REAL)omegaP;
    REAL *E = (REAL *)calloc((size_t)(N + 1) * (N + 1), sizeof(REAL));
    REAL *V = (REAL *)calloc((size_t)N + 2, sizeof(REAL));
    if (!E || !V) {
        free(E); free(V);
        return -2;
    }
#define EE(u, v) E[(size_t)(u) * (N + 1) + (v)]
#define S2(a, ja, bb, jb) FN(dist2_)(R, P, (a) - 1, (ja) - 1, (bb) - 1, (jb) - 1, Lr)
    for (int v = 1; v <= N; ++v)
        for (int u = 1; u <= v; ++u) {
            REAL s = 0;
            for (int l = u; l <= v; ++l)
                for (int j = 1; j <= P - 1; ++j) s += S2(l, j + 1, l, j);
            for (int l = u; l <= v - 1; ++l) s += S2(l + 1, 1, l, P);
            s += S2(u, 1, v, P);
            EE(u, v) = k * s;
        }
    Vb_out[0] = 0;
    for (int u = 1; u <= N; ++u) {
        /* V[M] holds V^[u,M]; index M = u-1 .. N */
        V[u - 1] = 0;
        for (int M = u; M <= N; ++M) {
            REAL sh = V[M - 1] + EE(M, M);
            for (int kk = 2; kk <= M - u + 1; ++kk) {
                REAL t = V[M - kk] + EE(M - kk + 1, M);
                if (t < sh) sh = t;
            }
            REAL acc = 0;
            for (int kk = 1; kk <= M - u + 1; ++kk) acc += EXP(-b * (V[M - kk] + EE(M - kk + 1, M) - sh));
            V[M] = sh - LOG(acc / (REAL)M) / b;
        }
        Vb_out[u] = (double)V[N];
    }
#undef EE
#undef S2
    free(E); free(V);
    return 0;
}

#undef FN
#undef CAT
#undef CAT_
