/*
 * CPU ORACLE -- test infrastructure only.  Nothing in the product path may
 * link or call this file; only the tests, the smoke check and the benchmark's
 * CPU-baseline leg do.
 *
 * Plain FP64 definition of the O(a)-improved Wilson-Dirac operator with
 * SU(3) x U(1) links and C* boundary conditions in space, realised on the
 * x-doubled lattice (paper, section "Sign of the Pfaffian": the doublet
 * (psi, psi^C) with psi(x+L k) = psi^C(x) makes D a 24V x 24V matrix;
 * simulation setup section: SW terms for SU(3) and U(1), C* in space,
 * periodic in time).
 *
 * Conventions (the paper fixes only C = i g0 g2 in a chiral basis):
 *  - physical lattice T x L^3, coordinates (t,x1,x2,x3), mu = 0 is t;
 *  - x-doubled lattice: x1 in [0,2L); site index ((t*2L + x1)*L + x2)*L + x3;
 *  - tau(x) = x + L e1 (mod 2L) maps a site to its charge-conjugate copy;
 *  - C* wrap: leaving [0,L) in x2 or x3 also shifts x1 by L; x1 has period 2L;
 *    t is periodic with the fermion phase time_bc (+1 or -1) on wrapping hops;
 *  - link on the doubled lattice: U_e(x) = U(x) for x1 < L, conj(U(tau x))
 *    otherwise; theta_e likewise with a sign flip; quark link
 *    V = exp(i q theta_e) U_e;
 *  - chiral basis: g0 = [[0,-1],[-1,0]], gk = [[0,-i s_k],[i s_k,0]],
 *    g5 = g0 g1 g2 g3 = diag(1,1,-1,-1);
 *  - (D psi)(x) = (4+m0) psi(x) + SW(x) psi(x)
 *        - 1/2 sum_mu [ ph+ (1-g_mu) V(x,mu) psi(x+mu) + ph- (1+g_mu) V(x-mu,mu)^H psi(x-mu) ]
 *  - SW(x) = (i/4) sum_{mu,nu} s_{mu nu} (x) F_{mu nu}(x),  s_{mu nu} = (i/2)[g_mu,g_nu],
 *    F = c_su3 * (Q - Q^H)/8 + q c_u1 * (i/4) sum_leaves sin(theta_leaf) * 1_3,
 *    Q_{mu nu}(x) = sum of the four plaquette leaves at x in the (mu,nu) plane,
 *    each oriented mu first, then nu.
 *
 * Spinor layout: [site][spin 4][colour 3] complex double (interleaved re,im).
 * Gauge input: su3 [T][L][L][L][4][3][3] complex, theta [T][L][L][L][4] double.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

typedef struct {
    int T, L, time_bc;
} geom;

static long n_sites(const geom *g) { return 2L * g->T * g->L * g->L * g->L; }

static long site_index(const geom *g, int t, int x1, int x2, int x3) {
    return (((long)t * 2 * g->L + x1) * g->L + x2) * g->L + x3;
}

static void site_coords(const geom *g, long s, int c[4]) {
    c[3] = (int)(s % g->L); s /= g->L;
    c[2] = (int)(s % g->L); s /= g->L;
    c[1] = (int)(s % (2 * g->L)); s /= 2 * g->L;
    c[0] = (int)s;
}

/* Neighbour of x in direction mu, step +1 or -1, on the x-doubled C* lattice.
 * *wrap_t is set when the hop crosses the time boundary. */
static void neighbour(const geom *g, const int x[4], int mu, int step, int y[4], int *wrap_t) {
    int L = g->L;
    y[0] = x[0]; y[1] = x[1]; y[2] = x[2]; y[3] = x[3];
    *wrap_t = 0;
    if (mu == 0) {
        y[0] = x[0] + step;
        if (y[0] == g->T) { y[0] = 0; *wrap_t = 1; }
        if (y[0] < 0) { y[0] = g->T - 1; *wrap_t = 1; }
    } else if (mu == 1) {
        y[1] = (x[1] + step + 2 * L) % (2 * L);
    } else {
        y[mu] = x[mu] + step;
        if (y[mu] == L || y[mu] < 0) {
            y[mu] = (y[mu] + L) % L;
            y[1] = (x[1] + L) % (2 * L);
        }
    }
}

/* Doubled-lattice SU(3) link U_e(x,mu) and U(1) angle theta_e(x,mu). */
static void link_e(const geom *g, const double *su3, const double *theta, const int x[4], int mu,
                   cplx U[3][3], double *th) {
    int L = g->L;
    int mirror = x[1] >= L;
    int x1 = mirror ? x[1] - L : x[1];
    long p = (((long)x[0] * L + x1) * L + x[2]) * L + x[3];
    const double *u = su3 + (p * 4 + mu) * 18;
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            cplx z = u[(a * 3 + b) * 2] + I * u[(a * 3 + b) * 2 + 1];
            U[a][b] = mirror ? conj(z) : z;
        }
    *th = mirror ? -theta[p * 4 + mu] : theta[p * 4 + mu];
}

/* ---- gamma matrices -------------------------------------------------------- */
static cplx G[6][4][4]; /* G[0..3] = gamma_mu, G[4] = gamma_5, G[5] = identity */
static cplx SIGMA[4][4][4][4]; /* sigma_{mu nu} = (i/2)[g_mu, g_nu] */
static int gamma_ready = 0;

static void matmul4(cplx a[4][4], cplx b[4][4], cplx c[4][4]) {
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) {
            cplx s = 0;
            for (int k = 0; k < 4; k++) s += a[i][k] * b[k][j];
            c[i][j] = s;
        }
}

static void init_gamma(void) {
    if (gamma_ready) return;
    memset(G, 0, sizeof(G));
    /* Pauli matrices */
    cplx s[3][2][2] = {{{0, 1}, {1, 0}}, {{0, -I}, {I, 0}}, {{1, 0}, {0, -1}}};
    /* g0 = [[0,-1],[-1,0]] (2x2 blocks) */
    for (int i = 0; i < 2; i++) { G[0][i][2 + i] = -1; G[0][2 + i][i] = -1; }
    /* gk = [[0, -i s_k],[i s_k, 0]] */
    for (int k = 0; k < 3; k++)
        for (int i = 0; i < 2; i++)
            for (int j = 0; j < 2; j++) {
                G[k + 1][i][2 + j] = -I * s[k][i][j];
                G[k + 1][2 + i][j] = I * s[k][i][j];
            }
    cplx t1[4][4], t2[4][4];
    matmul4(G[0], G[1], t1);
    matmul4(t1, G[2], t2);
    matmul4(t2, G[3], G[4]);
    for (int i = 0; i < 4; i++) G[5][i][i] = 1;
    for (int mu = 0; mu < 4; mu++)
        for (int nu = 0; nu < 4; nu++) {
            cplx a[4][4], b[4][4];
            matmul4(G[mu], G[nu], a);
            matmul4(G[nu], G[mu], b);
            for (int i = 0; i < 4; i++)
                for (int j = 0; j < 4; j++) SIGMA[mu][nu][i][j] = 0.5 * I * (a[i][j] - b[i][j]);
        }
    gamma_ready = 1;
}

/* ---- 3x3 helpers -------------------------------------------------------- */
static void mm3(cplx a[3][3], cplx b[3][3], cplx c[3][3]) {
    cplx r[3][3];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            cplx s = 0;
            for (int k = 0; k < 3; k++) s += a[i][k] * b[k][j];
            r[i][j] = s;
        }
    memcpy(c, r, sizeof(r));
}
static void dag3(cplx a[3][3], cplx c[3][3]) {
    cplx r[3][3];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) r[i][j] = conj(a[j][i]);
    memcpy(c, r, sizeof(r));
}

/* Path of links starting at x: steps[k] = +-(mu+1).  Returns the ordered
 * product of the traversed links (forward hop: U_e(y,mu); backward hop:
 * U_e(y-mu,mu)^H) and the oriented sum of the U(1) angles. */
static void path_product(const geom *g, const double *su3, const double *theta, const int x[4],
                         const int *steps, int nsteps, cplx P[3][3], double *phase) {
    int y[4] = {x[0], x[1], x[2], x[3]};
    int wrap;
    memset(P, 0, sizeof(cplx) * 9);
    P[0][0] = P[1][1] = P[2][2] = 1;
    *phase = 0;
    for (int k = 0; k < nsteps; k++) {
        int mu = abs(steps[k]) - 1;
        cplx U[3][3];
        double th;
        int z[4];
        if (steps[k] > 0) {
            link_e(g, su3, theta, y, mu, U, &th);
            neighbour(g, y, mu, +1, z, &wrap);
            *phase += th;
        } else {
            neighbour(g, y, mu, -1, z, &wrap);
            link_e(g, su3, theta, z, mu, U, &th);
            dag3(U, U);
            *phase -= th;
        }
        mm3(P, U, P);
        memcpy(y, z, sizeof(y));
    }
}

/*
 * Field strength per doubled site, F[site][plane][3][3] complex, plane index
 * p over (mu,nu) = (0,1),(0,2),(0,3),(1,2),(1,3),(2,3):
 *   F = c_su3 (Q - Q^H)/8 + q c_u1 (i/4) sum_leaves sin(theta_leaf) 1_3.
 * The four leaves in the (mu,nu) plane at x, each a closed loop from x:
 *   (+mu,+nu,-mu,-nu), (+nu,-mu,-nu,+mu), (-mu,-nu,+mu,+nu), (-nu,+mu,+nu,-mu).
 */
int oracle_field_strength(int T, int L, const double *su3, const double *theta, double q,
                          double csw_su3, double csw_u1, double *F_out) {
    geom g = {T, L, 1};
    long n = n_sites(&g);
    static const int planes[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
#pragma omp parallel for schedule(static)
    for (long s = 0; s < n; s++) {
        int x[4];
        site_coords(&g, s, x);
        for (int p = 0; p < 6; p++) {
            int a = planes[p][0] + 1, b = planes[p][1] + 1;
            int leaves[4][4] = {{a, b, -a, -b}, {b, -a, -b, a}, {-a, -b, a, b}, {-b, a, b, -a}};
            cplx Qm[3][3] = {{0}};
            double sin_sum = 0;
            for (int l = 0; l < 4; l++) {
                cplx P[3][3];
                double ph;
                path_product(&g, su3, theta, x, leaves[l], 4, P, &ph);
                for (int i = 0; i < 3; i++)
                    for (int j = 0; j < 3; j++) Qm[i][j] += P[i][j];
                sin_sum += sin(ph);
            }
            double *f = F_out + ((s * 6 + p) * 9) * 2;
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) {
                    cplx v = csw_su3 * (Qm[i][j] - conj(Qm[j][i])) / 8.0;
                    if (i == j) v += q * csw_u1 * (I * 0.25 * sin_sum);
                    f[(i * 3 + j) * 2] = creal(v);
                    f[(i * 3 + j) * 2 + 1] = cimag(v);
                }
        }
    }
    return 0;
}

/* BF16 rounding of a value: first to the nearest FP32, then round-to-nearest-even
 * to the 8 high mantissa bits of FP32 (the bfloat16 format). */
static double to_bf16(double v) {
    float f = (float)v;
    uint32_t u;
    memcpy(&u, &f, 4);
    uint32_t lsb = (u >> 16) & 1u;
    u = (u + 0x7FFFu + lsb) & 0xFFFF0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

/*
 * Quark link table on the doubled lattice, Vtab[site][mu][3][3] complex.
 * link_mode 0: V = exp(i q theta_e) U_e in FP64.
 * link_mode 1/2: the compressed formats -- rows 0 and 1 of the physical SU(3)
 *   link rounded to FP32 (1) or BF16 (2), row 2 = conj(row0 x row1), the
 *   quark phase exp(i q theta) stored as its cosine and sine each rounded to
 *   FP32; the mirror copy is the complex conjugate of the physical one.
 *   Arithmetic stays FP64.
 */
static void build_links(const geom *g, const double *su3, const double *theta, double q,
                        int link_mode, cplx *Vtab) {
    long n = n_sites(g);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < n; s++) {
        int x[4];
        site_coords(g, s, x);
        for (int mu = 0; mu < 4; mu++) {
            cplx U[3][3];
            double th;
            cplx *V = Vtab + (s * 4 + mu) * 9;
            if (link_mode == 0) {
                link_e(g, su3, theta, x, mu, U, &th);
                cplx ph = cexp(I * q * th);
                for (int i = 0; i < 3; i++)
                    for (int j = 0; j < 3; j++) V[i * 3 + j] = ph * U[i][j];
            } else {
                int mirror = x[1] >= g->L;
                int xp[4] = {x[0], mirror ? x[1] - g->L : x[1], x[2], x[3]};
                link_e(g, su3, theta, xp, mu, U, &th); /* physical link */
                cplx R[3][3];
                for (int i = 0; i < 2; i++)
                    for (int j = 0; j < 3; j++) {
                        double re = creal(U[i][j]), im = cimag(U[i][j]);
                        if (link_mode == 1) { re = (double)(float)re; im = (double)(float)im; }
                        else { re = to_bf16(re); im = to_bf16(im); }
                        R[i][j] = re + I * im;
                    }
                R[2][0] = conj(R[0][1] * R[1][2] - R[0][2] * R[1][1]);
                R[2][1] = conj(R[0][2] * R[1][0] - R[0][0] * R[1][2]);
                R[2][2] = conj(R[0][0] * R[1][1] - R[0][1] * R[1][0]);
                double phi = q * th;
                cplx ph = (double)(float)cos(phi) + I * (double)(float)sin(phi);
                for (int i = 0; i < 3; i++)
                    for (int j = 0; j < 3; j++) {
                        cplx v = ph * R[i][j];
                        V[i * 3 + j] = mirror ? conj(v) : v;
                    }
            }
        }
    }
}

/*
 * The quark link table as the operator uses it, for the oracle's own pins:
 * Vtab_out[site][mu][3][3] complex double on the doubled lattice (link_mode
 * as in build_links).
 */
int oracle_links(int T, int L, double q, const double *su3, const double *theta, int link_mode, double *Vtab_out) {
    geom g = {T, L, 1};
    build_links(&g, su3, theta, q, link_mode, (cplx *)Vtab_out);
    return 0;
}

/*
 * out = D(m0) in   (gamma5 != 0: out = gamma5 D(m0) in) with a link table
 * from oracle_links.  F: field strength from oracle_field_strength (NULL: no
 * clover term).  in/out: [2V][4][3] complex double, non-aliasing.
 */
int oracle_dirac_tab(int T, int L, int time_bc, const double *Vtab_in, const double *F, double m0, int gamma5,
                     const double *in, double *out) {
    init_gamma();
    geom g = {T, L, time_bc};
    long n = n_sites(&g);
    const cplx *Vtab = (const cplx *)Vtab_in;
    const cplx *psi = (const cplx *)in;
    cplx *res = (cplx *)out;
    static const int planes[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
#pragma omp parallel for schedule(static)
    for (long s = 0; s < n; s++) {
        int x[4];
        site_coords(&g, s, x);
        cplx acc[4][3];
        /* mass + Wilson diagonal */
        for (int a = 0; a < 4; a++)
            for (int c = 0; c < 3; c++) acc[a][c] = (4.0 + m0) * psi[s * 12 + a * 3 + c];
        /* clover: (i/4) sum_{mu,nu} sigma_{mu nu} F_{mu nu} = (i/2) sum_{mu<nu} */
        if (F) {
            for (int p = 0; p < 6; p++) {
                int mu = planes[p][0], nu = planes[p][1];
                const double *f = F + ((s * 6 + p) * 9) * 2;
                cplx Fc[3][3];
                for (int i = 0; i < 3; i++)
                    for (int j = 0; j < 3; j++) Fc[i][j] = f[(i * 3 + j) * 2] + I * f[(i * 3 + j) * 2 + 1];
                cplx tmp[4][3];
                for (int a = 0; a < 4; a++)
                    for (int i = 0; i < 3; i++) {
                        cplx v = 0;
                        for (int j = 0; j < 3; j++) v += Fc[i][j] * psi[s * 12 + a * 3 + j];
                        tmp[a][i] = v;
                    }
                for (int a = 0; a < 4; a++)
                    for (int b = 0; b < 4; b++) {
                        cplx sab = 0.5 * I * SIGMA[mu][nu][a][b];
                        if (sab == 0) continue;
                        for (int i = 0; i < 3; i++) acc[a][i] += sab * tmp[b][i];
                    }
            }
        }
        /* hopping */
        for (int mu = 0; mu < 4; mu++) {
            for (int dir = 0; dir < 2; dir++) {
                int y[4], wrap;
                neighbour(&g, x, mu, dir == 0 ? +1 : -1, y, &wrap);
                long sy = site_index(&g, y[0], y[1], y[2], y[3]);
                double ph = wrap ? (double)time_bc : 1.0;
                cplx W[3][3];
                if (dir == 0) {
                    const cplx *V = Vtab + (s * 4 + mu) * 9;
                    for (int i = 0; i < 3; i++)
                        for (int j = 0; j < 3; j++) W[i][j] = V[i * 3 + j];
                } else {
                    const cplx *V = Vtab + (sy * 4 + mu) * 9;
                    for (int i = 0; i < 3; i++)
                        for (int j = 0; j < 3; j++) W[i][j] = conj(V[j * 3 + i]);
                }
                /* chi = W psi(y) (colour), then (1 -/+ g_mu) on spin */
                cplx chi[4][3];
                for (int a = 0; a < 4; a++)
                    for (int i = 0; i < 3; i++) {
                        cplx v = 0;
                        for (int j = 0; j < 3; j++) v += W[i][j] * psi[sy * 12 + a * 3 + j];
                        chi[a][i] = v;
                    }
                double sg = dir == 0 ? -1.0 : 1.0;
                for (int a = 0; a < 4; a++)
                    for (int b = 0; b < 4; b++) {
                        cplx pr = (a == b ? 1.0 : 0.0) + sg * G[mu][a][b];
                        if (pr == 0) continue;
                        for (int i = 0; i < 3; i++) acc[a][i] -= 0.5 * ph * pr * chi[b][i];
                    }
            }
        }
        for (int a = 0; a < 4; a++)
            for (int i = 0; i < 3; i++) {
                cplx v = acc[a][i];
                if (gamma5) {
                    cplx w = 0;
                    for (int b = 0; b < 4; b++) w += G[4][a][b] * acc[b][i];
                    v = w;
                }
                res[s * 12 + a * 3 + i] = v;
            }
    }
    return 0;
}

/* As oracle_dirac_tab, building the link table for this call. */
int oracle_dirac(int T, int L, int time_bc, double q, const double *su3, const double *theta,
                 const double *F, double m0, int gamma5, int link_mode, const double *in, double *out) {
    geom g = {T, L, time_bc};
    long n = n_sites(&g);
    cplx *Vtab = (cplx *)malloc(sizeof(cplx) * n * 36);
    if (!Vtab) return -2;
    build_links(&g, su3, theta, q, link_mode, Vtab);
    int rc = oracle_dirac_tab(T, L, time_bc, (const double *)Vtab, F, m0, gamma5, in, out);
    free(Vtab);
    return rc;
}

/*
 * Site-local part of D on every doubled site (it is what D keeps when it is
 * restricted to one parity of sites, as in the even-odd decomposition of the
 * mass-reweighting section):
 *   out[s][a*3+i][b*3+j] = (4+m0) delta_ab delta_ij + (i/2) sum_{mu<nu} sigma_{mu nu}[a][b] F_{mu nu}(s)[i][j],
 * complex double; F from oracle_field_strength (NULL: no clover term).
 */
int oracle_local_term(int T, int L, const double *F, double m0, double *out) {
    init_gamma();
    geom g = {T, L, 1};
    long n = n_sites(&g);
    static const int planes[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
#pragma omp parallel for schedule(static)
    for (long s = 0; s < n; s++) {
        cplx M[12][12];
        for (int r = 0; r < 12; r++)
            for (int c = 0; c < 12; c++) M[r][c] = (r == c) ? (4.0 + m0) : 0.0;
        if (F) {
            for (int p = 0; p < 6; p++) {
                int mu = planes[p][0], nu = planes[p][1];
                const double *f = F + ((s * 6 + p) * 9) * 2;
                for (int a = 0; a < 4; a++)
                    for (int b = 0; b < 4; b++) {
                        cplx sab = 0.5 * I * SIGMA[mu][nu][a][b];
                        if (sab == 0) continue;
                        for (int i = 0; i < 3; i++)
                            for (int j = 0; j < 3; j++)
                                M[a * 3 + i][b * 3 + j] += sab * (f[(i * 3 + j) * 2] + I * f[(i * 3 + j) * 2 + 1]);
                    }
            }
        }
        double *o = out + s * 288;
        for (int r = 0; r < 12; r++)
            for (int c = 0; c < 12; c++) {
                o[(r * 12 + c) * 2] = creal(M[r][c]);
                o[(r * 12 + c) * 2 + 1] = cimag(M[r][c]);
            }
    }
    return 0;
}

/* Gamma matrices as used above (for the oracle's own self-tests):
 * out[6][4][4] complex = g0,g1,g2,g3,g5,1. */
void oracle_gammas(double *out) {
    init_gamma();
    for (int k = 0; k < 6; k++)
        for (int i = 0; i < 4; i++)
            for (int j = 0; j < 4; j++) {
                out[((k * 4 + i) * 4 + j) * 2] = creal(G[k][i][j]);
                out[((k * 4 + i) * 4 + j) * 2 + 1] = cimag(G[k][i][j]);
            }
}

/* C* neighbour map exported for the oracle's tests: idx_out[site][8] with
 * entries for (mu, +1), (mu, -1), mu = 0..3. */
void oracle_neighbours(int T, int L, long *idx_out) {
    geom g = {T, L, 1};
    long n = n_sites(&g);
    for (long s = 0; s < n; s++) {
        int x[4], y[4], w;
        site_coords(&g, s, x);
        for (int mu = 0; mu < 4; mu++)
            for (int d = 0; d < 2; d++) {
                neighbour(&g, x, mu, d ? -1 : 1, y, &w);
                idx_out[s * 8 + mu * 2 + d] = site_index(&g, y[0], y[1], y[2], y[3]);
            }
    }
}

/*
 * Parallel transport used by the gauge-covariant network (oracle side):
 *   dir = +1: out(x) = ph * V(x,mu) psi(x+mu),   dir = -1: out(x) = ph * V(x-mu,mu)^H psi(x-mu),
 * colour only (the same 3x3 acts on every spin), ph = time_bc on hops that wrap
 * in time, V the quark link on the doubled lattice (link_mode as in oracle_dirac).
 */
int oracle_transport(int T, int L, int time_bc, double q, const double *su3, const double *theta, int mu,
                     int dir, int link_mode, const double *in, double *out) {
    geom g = {T, L, time_bc};
    long n = n_sites(&g);
    cplx *Vtab = (cplx *)malloc(sizeof(cplx) * n * 36);
    if (!Vtab) return -2;
    build_links(&g, su3, theta, q, link_mode, Vtab);
    const cplx *psi = (const cplx *)in;
    cplx *res = (cplx *)out;
#pragma omp parallel for schedule(static)
    for (long s = 0; s < n; s++) {
        int x[4], y[4], wrap;
        site_coords(&g, s, x);
        neighbour(&g, x, mu, dir, y, &wrap);
        long sy = site_index(&g, y[0], y[1], y[2], y[3]);
        double ph = wrap ? (double)time_bc : 1.0;
        cplx W[3][3];
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++)
                W[i][j] = dir > 0 ? Vtab[(s * 4 + mu) * 9 + i * 3 + j] : conj(Vtab[(sy * 4 + mu) * 9 + j * 3 + i]);
        for (int a = 0; a < 4; a++)
            for (int i = 0; i < 3; i++) {
                cplx v = 0;
                for (int j = 0; j < 3; j++) v += W[i][j] * psi[sy * 12 + a * 3 + j];
                res[s * 12 + a * 3 + i] = ph * v;
            }
    }
    free(Vtab);
    return 0;
}
