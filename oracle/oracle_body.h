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
 * Fast PIMD-B (Alg. 1 of the paper's appendix "Algorithm Pseudocode"),
 * taken step by step in the paper's order:
 *   1. interior spring energies E_int (Theory, "Reducing the potential",
 *      definition of E_int: springs j = 1..P-1, j = P excluded);
 *   2. cycle energies E^[u,v]: single-particle base case E^[v,v], then the
 *      incremental break-and-reform recurrence in u (same subsection);
 *   3. forward potentials V^[1,v] by the recurrence over the length of the
 *      cycle containing v (Background, recurrence for V^[1,N]), stabilised
 *      by the shift of the appendix "Numerical Stability";
 *   4. backward potentials V^[u,N] (Theory, "Connection probabilities",
 *      backward recursion with the 1/l weight on the absolute end index);
 *   5. connection probabilities: direct link Pr[l -> l+1] and cycle closing
 *      Pr[l -> u], u <= l (Methods, "Expressions for connection
 *      probabilities"); zero for u > l+1 (appendix lemma on vanishing
 *      probabilities);
 *   6. interior bead forces (Theory, "Force on interior beads");
 *   7. exterior bead forces (Theory, "Force on exterior beads") with the
 *      summation limits of Alg. 1, clamped to 1..N.
 *
 * shift_mode 0: the shift is the minimum over the terms (largest exponent
 * zero), the choice the paper uses for large systems.  shift_mode 1: the
 * simpler two-term shift the paper describes for small trapped systems.
 * Every shift is exact in exact arithmetic; they differ only in rounding
 * and in overflow behaviour.
 *
 * Outputs (all optional except V): V = V^[1,N]; F = -grad V in the
 * oracle layout; Vf[0..N] = V^[1,v]; Vb[0..N+1] with Vb[u] = V^[u,N] for
 * u = 1..N+1 (Vb[0] unused, set to 0); Pr[(l-1)*N + (l'-1)] = Pr[l -> l'];
 * E[(u-1)*N + (v-1)] = E^[u,v] for u <= v (0 elsewhere); Eint[l-1].
 * Returns 0, or -1 on invalid arguments, -2 on allocation failure.
 */
int FN(orc_alg1)(int N, int P, const double *R, double beta, double m, double omegaP, double L,
                 int shift_mode, double *V_out, double *F_out, double *Vf_out, double *Vb_out,
                 double *Pr_out, double *E_out, double *Eint_out) {
    if (N < 1 || P < 2 || !(beta > 0) || !(m > 0) || !(omegaP > 0) || !(L >= 0) || !R || !V_out)
        return -1;
    const REAL b = (REAL)beta;
    const REAL Lr = (REAL)L;
    const REAL k = (REAL)0.5 * (REAL)m * (REAL)omegaP * (REAL)omegaP;
    const REAL mw2 = (REAL)m * (REAL)omegaP * (REAL)omegaP;

    REAL *Eint = (REAL *)calloc((size_t)N + 1, sizeof(REAL));          /* 1-based */
    REAL *E = (REAL *)calloc((size_t)(N + 1) * (N + 1), sizeof(REAL)); /* E[u*(N+1)+v] */
    REAL *Vf = (REAL *)calloc((size_t)N + 1, sizeof(REAL));
    REAL *Vb = (REAL *)calloc((size_t)N + 2, sizeof(REAL));
    REAL *Pr = (REAL *)calloc((size_t)(N + 2) * (N + 2), sizeof(REAL)); /* Pr[l*(N+2)+l'] */
    REAL *terms = (REAL *)calloc((size_t)N + 1, sizeof(REAL));
    if (!Eint || !E || !Vf || !Vb || !Pr || !terms) {
        free(Eint); free(E); free(Vf); free(Vb); free(Pr); free(terms);
        return -2;
    }
#define EE(u, v) E[(size_t)(u) * (N + 1) + (v)]
#define PR(l, lp) Pr[(size_t)(l) * (N + 2) + (lp)]
    /* particle l (1-based) bead j (1-based) -> 0-based indices */
#define S2(a, ja, bb, jb) FN(dist2_)(R, P, (a) - 1, (ja) - 1, (bb) - 1, (jb) - 1, Lr)

    /* 1. interior energies */
    for (int l = 1; l <= N; ++l) {
        REAL s = 0;
        for (int j = 1; j <= P - 1; ++j) s += S2(l, j + 1, l, j);
        Eint[l] = k * s;
    }
    /* 2. cycle energies */
    for (int v = 1; v <= N; ++v) {
        EE(v, v) = Eint[v] + k * S2(v, P, v, 1);
        for (int u = v - 1; u >= 1; --u) {
            EE(u, v) = EE(u + 1, v) - k * S2(v, P, u + 1, 1) + k * S2(u, P, u + 1, 1) + Eint[u] +
                       k * S2(v, P, u, 1);
        }
    }
    /* 3. forward potentials V^[1,v], v = 1..N, V^[1,0] = 0 */
    Vf[0] = 0;
    for (int v = 1; v <= N; ++v) {
        /* term for cycle length kk: V^[1,v-kk] + E^[v-kk+1, v] */
        for (int kk = 1; kk <= v; ++kk) terms[kk] = Vf[v - kk] + EE(v - kk + 1, v);
        REAL sh;
        if (shift_mode == 1) {
            /* two-term shift: min(E^[1,v], V^[1,v-1] + E^[v,v]) */
            sh = EE(1, v);
            REAL t = Vf[v - 1] + EE(v, v);
            if (t < sh) sh = t;
        } else {
            sh = terms[1];
            for (int kk = 2; kk <= v; ++kk)
                if (terms[kk] < sh) sh = terms[kk];
        }
        REAL acc = 0;
        for (int kk = 1; kk <= v; ++kk) acc += EXP(-b * (terms[kk] - sh));
        Vf[v] = sh - LOG(acc / (REAL)v) / b;
    }
    /* 4. backward potentials V^[u,N], u = N..1, V^[N+1,N] = 0 */
    Vb[N + 1] = 0;
    for (int u = N; u >= 1; --u) {
        for (int l = u; l <= N; ++l) terms[l] = EE(u, l) + Vb[l + 1];
        REAL sh;
        if (shift_mode == 1) {
            /* two-term shift: min(E^[u,u] + V^[u+1,N], E^[u,N]) */
            sh = EE(u, u) + Vb[u + 1];
            if (EE(u, N) < sh) sh = EE(u, N);
        } else {
            sh = terms[u];
            for (int l = u + 1; l <= N; ++l)
                if (terms[l] < sh) sh = terms[l];
        }
        REAL acc = 0;
        for (int l = u; l <= N; ++l) acc += EXP(-b * (terms[l] - sh)) / (REAL)l;
        Vb[u] = sh - LOG(acc) / b;
    }
    const REAL VN = Vf[N];
    /* 5. connection probabilities */
    for (int l = 1; l <= N - 1; ++l) PR(l, l + 1) = -EXPM1(-b * (Vf[l] + Vb[l + 1] - VN));
    for (int lp = 1; lp <= N; ++lp)
        for (int l = lp; l <= N; ++l)
            PR(l, lp) = EXP(-b * (Vf[lp - 1] + EE(lp, l) + Vb[l + 1] - VN)) / (REAL)l;

    if (F_out) {
        /* 6. interior beads j = 2..P-1 */
        for (int l = 1; l <= N; ++l) {
            for (int j = 2; j <= P - 1; ++j) {
                REAL d1[3], d2[3];
                FN(disp_)(R, P, l - 1, j - 1, l - 1, j - 2, Lr, d1); /* r^j - r^{j-1} */
                FN(disp_)(R, P, l - 1, j - 1, l - 1, j, Lr, d2);     /* r^j - r^{j+1} */
                for (int c = 0; c < 3; ++c)
                    F_out[(((size_t)l - 1) * P + (j - 1)) * 3 + c] = (double)(-mw2 * (d1[c] + d2[c]));
            }
        }
        /* 7. exterior beads: j = 1 sums over predecessors l' (Pr[l' -> l]),
         *    j = P sums over successors l' (Pr[l -> l']). */
        for (int l = 1; l <= N; ++l) {
            REAL f1[3] = {0, 0, 0}, fP[3] = {0, 0, 0};
            int lo = l - 1 < 1 ? 1 : l - 1;
            for (int lp = lo; lp <= N; ++lp) {
                REAL pr = PR(lp, l);
                REAL a[3], bb[3];
                FN(disp_)(R, P, l - 1, 0, l - 1, 1, Lr, a);       /* r_l^1 - r_l^2 */
                FN(disp_)(R, P, l - 1, 0, lp - 1, P - 1, Lr, bb); /* r_l^1 - r_l'^P */
                for (int c = 0; c < 3; ++c) f1[c] += pr * mw2 * (a[c] + bb[c]);
            }
            int hi = l + 1 > N ? N : l + 1;
            for (int lp = 1; lp <= hi; ++lp) {
                REAL pr = PR(l, lp);
                REAL a[3], bb[3];
                FN(disp_)(R, P, l - 1, P - 1, l - 1, P - 2, Lr, a); /* r_l^P - r_l^{P-1} */
                FN(disp_)(R, P, l - 1, P - 1, lp - 1, 0, Lr, bb);   /* r_l^P - r_l'^1 */
                for (int c = 0; c < 3; ++c) fP[c] += pr * mw2 * (a[c] + bb[c]);
            }
            for (int c = 0; c < 3; ++c) {
                F_out[(((size_t)l - 1) * P + 0) * 3 + c] = (double)(-f1[c]);
                F_out[(((size_t)l - 1) * P + (P - 1)) * 3 + c] = (double)(-fP[c]);
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
    free(Eint); free(E); free(Vf); free(Vb); free(Pr); free(terms);
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
