/*
 * lbfd_oracle.c -- plain, slow, FP64 CPU oracle of one time step of the hybrid
 * lattice-Boltzmann / finite-difference method of Gupta, Sbragaglia & Scagliarini,
 * "Hybrid Lattice Boltzmann/Finite Difference simulations of viscoelastic
 * multicomponent flows in confined geometries" (arXiv:1406.2686).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file; it exists so that tests, the smoke check and the CPU baseline of the
 * benchmark can judge the GPU library.  It shares no code, header, table or
 * helper with the GPU library.
 *
 * What it computes (one step, Jacobi in time: every stage reads level n only):
 *   S1  moments: rho_s = sum_a f_sa, j = sum_s sum_a c_a f_sa        (Sec. 2, moments eq.)
 *   S2  order parameter phi = (rho_A - rho_B)/rho and
 *       f+-(phi) = (1 +- tanh(phi/Delta))/2                          (Sec. 2, eq. smoothingvisco)
 *   S3  Shan-Chen force g_s = -G rho_s sum_a w_a rho_s'(x + c_a) c_a  (Sec. 2, eq. SCforce)
 *   S4  polymer stress T = (eta_P/tau_P) m(phi) (f(r) C - I),
 *       f(r) = (L^2 - 3)/(L^2 - tr C), and its divergence by 2nd-order central
 *       differences F_p,j = sum_i d_i T_ij                          (Sec. 2, FENE-P feedback;
 *                                                                     modulated-feedback eq.)
 *   S5  force split F_s = g_s + (rho_s/rho) F_p (species weight of eq. MODEtransformation);
 *       with the stress coupling instead F_s = g_s and T_s = (rho_s/rho) T lowers the
 *       second moment of the equilibrium in S8 (eq. MODEtransformation)
 *   S6  velocity u = (j + sum_s F_s / 2)/rho                          (Sec. 2, eq. equilibrium:vel)
 *   S7  local BGK time tau = tau_B + (tau_A - tau_B) f+(phi)
 *   S8  BGK collision with the equilibrium and source of Sec. 2 (eq. LB with Lambda = I/tau);
 *       or, as an option, the multiple-relaxation-time collision of Sec. 2: moments
 *       m = T f in an orthogonal D3Q19 basis, the bulk and shear modes relaxed with
 *       1/tau (tau_s = tau_b = the local tau), the species momentum with 1/tau_M = 1 and
 *       every other mode with rate 1 (eq. TRANSPORTCOEFF and the text after it), the
 *       source weighted by (I - Lambda/2) in moment space
 *   S9  streaming; half-way bounce-back with the moving-wall correction at y walls
 *   S10 FENE-P: C += dt [ -(u.grad)_upwind C + G^T C + C G - (f C - I)/tau_P ],
 *       G_ij = d_i u_j (central), dt = 1                              (Sec. 2, eq. FENE);
 *       or, as an option, the paper's integrator (Sec. 2, paragraph on the FENE-P solver):
 *       sigma_P = f C = L L^t evolved through the Cholesky factor L with ln l_ii in place
 *       of l_ii, second-order central differences in space, an artificial diffusivity
 *       kappa lap C, and second-order Adams-Bashforth in time
 *   S11 fault checks (non-finite, tr C >= L^2, non-positive leading minor); never clips.
 *
 * Readings where the paper is silent (all listed in the design notes): BGK instead of
 * MRT; polymer stress fed back as a body force; C stored and evolved directly with
 * first-order upwind advection and forward Euler; Shan-Chen and order-parameter
 * neighbours across a wall copy the wall-adjacent layer (neutral wetting); C ghosts by
 * linear extrapolation (Sec. 2, last paragraph on the FENE-P boundary condition);
 * velocity ghosts by reflection through the wall velocity.
 *
 * Arithmetic: IEEE binary64, compiled with -ffp-contract=off; every loop runs in
 * fixed z, y, x, alpha order; OpenMP only splits pure per-node maps over z, and all
 * reductions are serial, so results do not depend on the thread count.
 *
 * Layout: node n = (z*ny + y)*nx + x; populations f[(s*19 + a)*N + n];
 * symmetric tensors [k*N + n] with k = (xx, yy, zz, xy, xz, yz).
 */
#define _USE_MATH_DEFINES
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NQ 19

/* D3Q19 velocity set; opposite directions are adjacent (a, a+1) for a >= 1.
 * Weights 1/3, 1/18, 1/36 as printed in Sec. 2 (D3Q19 weights). */
static const int CX[NQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int CY[NQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int CZ[NQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
static const int OPP[NQ] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};

static double W(int a) { return a == 0 ? 1.0 / 3.0 : (a <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }

/* fault flags */
#define ORC_F_NONFINITE 1
#define ORC_F_EXTENSIBILITY 2
#define ORC_F_NOT_SPD 4

/* polymer phase selector for the feedback modulation m(phi) */
#define ORC_PHASE_NONE 0
#define ORC_PHASE_A 1
#define ORC_PHASE_B 2
#define ORC_PHASE_ALL 3

/* how the polymer stress reaches the fluid */
#define ORC_COUPLING_FORCE 0  /* body force F_p = div T, split by rho_s/rho (Sec. 2, eq. NS) */
#define ORC_COUPLING_STRESS 1 /* T_s = (rho_s/rho) T subtracted from the equilibrium's second
                                 moment (Sec. 2, eq. MODEtransformation) */

/* collision operator */
#define ORC_COLLISION_BGK 0
#define ORC_COLLISION_MRT 1

/* FENE-P integrator */
#define ORC_FENE_UPWIND_EULER 0
#define ORC_FENE_CHOLESKY_AB2 1

typedef struct {
    int nx, ny, nz, nc;
    long N;
    double tauA, tauB, G, delta, eta_p, tau_p, L2;
    int phase;
    int coupling;
    int collision;
    int fene;         /* ORC_FENE_* */
    double kappa;     /* artificial diffusivity of the Cholesky scheme */
    double *Hp, *Hn;  /* [6][N] rate of (ln l11, l21, ln l22, l31, l32, ln l33) at the last step */
    int have_hist;    /* Hp holds the previous rate (else the step is forward Euler) */
    double ub[3], ut[3];
    double *f, *fn;   /* [nc][19][N] */
    double *C, *Cn;   /* [6][N]      */
    double *rho;      /* [nc][N]     */
    double *j;        /* [3][N]      */
    double *phi;      /* [N]         */
    double *g;        /* [nc][3][N]  */
    double *Fp;       /* [3][N]      */
    double *F;        /* [nc][3][N]  */
    double *u;        /* [3][N]      */
    double *tau;      /* [N]         */
    long steps;
    int flags;
} orc_t;

static long IDX(const orc_t *o, int x, int y, int z) { return ((long)z * o->ny + y) * o->nx + x; }
static int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }
static int clampy(const orc_t *o, int y) { return y < 0 ? 0 : (y >= o->ny ? o->ny - 1 : y); }
static int sym(int i, int j) {
    if (i == j) return i;
    int s = i + j;
    return s == 1 ? 3 : (s == 2 ? 4 : 5);
}

/* ------------------------------------------------------------------ lifecycle */

orc_t *orc_create(int nx, int ny, int nz, int nc) {
    if (nx < 1 || ny < 3 || nz < 1 || (nc != 1 && nc != 2)) return NULL;
    orc_t *o = (orc_t *)calloc(1, sizeof(orc_t));
    o->nx = nx; o->ny = ny; o->nz = nz; o->nc = nc;
    o->N = (long)nx * ny * nz;
    long N = o->N;
    o->f = (double *)calloc((size_t)nc * NQ * N, sizeof(double));
    o->fn = (double *)calloc((size_t)nc * NQ * N, sizeof(double));
    o->C = (double *)calloc((size_t)6 * N, sizeof(double));
    o->Cn = (double *)calloc((size_t)6 * N, sizeof(double));
    o->rho = (double *)calloc((size_t)nc * N, sizeof(double));
    o->j = (double *)calloc((size_t)3 * N, sizeof(double));
    o->phi = (double *)calloc((size_t)N, sizeof(double));
    o->g = (double *)calloc((size_t)nc * 3 * N, sizeof(double));
    o->Fp = (double *)calloc((size_t)3 * N, sizeof(double));
    o->F = (double *)calloc((size_t)nc * 3 * N, sizeof(double));
    o->u = (double *)calloc((size_t)3 * N, sizeof(double));
    o->tau = (double *)calloc((size_t)N, sizeof(double));
    o->Hp = (double *)calloc((size_t)6 * N, sizeof(double));
    o->Hn = (double *)calloc((size_t)6 * N, sizeof(double));
    o->tauA = o->tauB = 1.0;
    o->delta = 0.1;
    o->L2 = 100.0;
    o->tau_p = 1000.0;
    o->phase = ORC_PHASE_NONE;
    return o;
}

void orc_destroy(orc_t *o) {
    if (!o) return;
    free(o->f); free(o->fn); free(o->C); free(o->Cn); free(o->rho); free(o->j);
    free(o->phi); free(o->g); free(o->Fp); free(o->F); free(o->u); free(o->tau);
    free(o->Hp); free(o->Hn);
    free(o);
}

void orc_set_params(orc_t *o, double tauA, double tauB, double G, double delta, int phase,
                    double eta_p, double tau_p, double L2, int coupling) {
    o->tauA = tauA; o->tauB = tauB; o->G = G; o->delta = delta; o->phase = phase;
    o->eta_p = eta_p; o->tau_p = tau_p; o->L2 = L2; o->coupling = coupling;
}

static void mrt_table(void);

void orc_set_fene(orc_t *o, int scheme, double kappa) {
    o->fene = scheme;
    o->kappa = kappa;
    o->have_hist = 0;
}

void orc_set_collision(orc_t *o, int collision) {
    o->collision = collision;
    if (collision == ORC_COLLISION_MRT) mrt_table(); /* before any parallel region reads it */
}

void orc_set_walls(orc_t *o, const double ub[3], const double ut[3]) {
    for (int d = 0; d < 3; d++) { o->ub[d] = ub[d]; o->ut[d] = ut[d]; }
}

long orc_steps(const orc_t *o) { return o->steps; }

/* ------------------------------------------------------- single-node formulas */

/* Equilibrium of Sec. 2: E_a = w_a rho [1 + c.u/cs2 + uu:(cc - cs2 I)/(2 cs2^2)], cs2 = 1/3. */
static double equilibrium(int a, double rho, const double u[3]) {
    double cu = CX[a] * u[0] + CY[a] * u[1] + CZ[a] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return W(a) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
}

/* Source term of Sec. 2: S_a = w_a [ (c - u)/cs2 + (c.u) c / cs2^2 ] . F. */
static double source(int a, const double u[3], const double F[3]) {
    double c[3] = {CX[a], CY[a], CZ[a]};
    double cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
    double s = 0.0;
    for (int d = 0; d < 3; d++) s += (3.0 * (c[d] - u[d]) + 9.0 * cu * c[d]) * F[d];
    return W(a) * s;
}

/* Polymer stress in the equilibrium (Sec. 2, eq. MODEtransformation): the second moment of
 * the equilibrium of species s is lowered by T_s.  With Q_a = c_a c_a - cs2 I the
 * D3Q19 fourth-order isotropy gives sum_a w_a c_a c_a (Q_a : T) = 2 cs2^2 T, so the term
 * -w_a Q_a : T_s / (2 cs2^2) = -4.5 w_a (c_a . T_s . c_a - tr T_s / 3) does exactly that and
 * leaves the zeroth and first moments unchanged.  T_s in (xx, yy, zz, xy, xz, yz) order. */
static double equilibrium_stress_term(int a, const double Ts[6]) {
    double c[3] = {CX[a], CY[a], CZ[a]};
    double cTc = c[0] * c[0] * Ts[0] + c[1] * c[1] * Ts[1] + c[2] * c[2] * Ts[2] +
                 2.0 * (c[0] * c[1] * Ts[3] + c[0] * c[2] * Ts[4] + c[1] * c[2] * Ts[5]);
    double tr = Ts[0] + Ts[1] + Ts[2];
    return -4.5 * W(a) * (cTc - tr / 3.0);
}

/* ------------------------------------------------------------------ MRT collision
 *
 * The paper names the moment basis of Premnath & Abraham (after d'Humieres et al.) without
 * printing it.  Reading: the 19 moments below, polynomials in c_a that are mutually
 * orthogonal over the 19 velocities (plain sum), in the usual order
 *   0 rho   1 e   2 eps   3 j_x  4 q_x  5 j_y  6 q_y  7 j_z  8 q_z
 *   9 3p_xx  10 3pi_xx  11 p_ww  12 pi_ww  13 p_xy  14 p_yz  15 p_xz  16 m_x  17 m_y  18 m_z.
 * Rates: e and the five stresses (9, 11, 13, 14, 15) relax with 1/tau (the paper's
 * tau_b = tau_s, space dependent through phi); the species momenta (3, 5, 7) with
 * 1/tau_M = 1; the non-hydrodynamic modes with 1; rho is conserved.  The collision is
 *   f* = f - T^-1 Lambda T (f - E) + T^-1 (I - Lambda/2) T S,
 * with T^-1 = T^t diag(1/|m_i|^2) because the rows are orthogonal (a pin checks it). */
static double mrt_row(int i, int a) {
    double x = CX[a], y = CY[a], z = CZ[a];
    double c2 = x * x + y * y + z * z;
    switch (i) {
        case 0: return 1.0;
        case 1: return 19.0 * c2 - 30.0;
        case 2: return (21.0 * c2 * c2 - 53.0 * c2 + 24.0) / 2.0;
        case 3: return x;
        case 4: return (5.0 * c2 - 9.0) * x;
        case 5: return y;
        case 6: return (5.0 * c2 - 9.0) * y;
        case 7: return z;
        case 8: return (5.0 * c2 - 9.0) * z;
        case 9: return 3.0 * x * x - c2;
        case 10: return (3.0 * c2 - 5.0) * (3.0 * x * x - c2);
        case 11: return y * y - z * z;
        case 12: return (3.0 * c2 - 5.0) * (y * y - z * z);
        case 13: return x * y;
        case 14: return y * z;
        case 15: return x * z;
        case 16: return (y * y - z * z) * x;
        case 17: return (z * z - x * x) * y;
        default: return (x * x - y * y) * z;
    }
}

static double mrt_rate(int i, double tau) {
    switch (i) {
        case 1: case 9: case 11: case 13: case 14: case 15: return 1.0 / tau; /* bulk, shear */
        default: return 1.0; /* rho (conserved), momenta (tau_M = 1), non-hydrodynamic */
    }
}

/* the basis as a table (filled once from mrt_row) and the squared row norms */
static double MRT_M[NQ][NQ], MRT_N2[NQ];
static void mrt_table(void) {
    static int done = 0;
    if (done) return;
    for (int i = 0; i < NQ; i++) {
        MRT_N2[i] = 0.0;
        for (int a = 0; a < NQ; a++) {
            MRT_M[i][a] = mrt_row(i, a);
            MRT_N2[i] += MRT_M[i][a] * MRT_M[i][a];
        }
    }
    done = 1;
}

/* f* at one node: f, E, S are the 19 populations, equilibrium and source. */
static void mrt_collide(const double *f, const double *E, const double *S, double tau, double *out) {
    double dm[NQ], sm[NQ];
    for (int i = 0; i < NQ; i++) {
        dm[i] = 0.0; sm[i] = 0.0;
        for (int a = 0; a < NQ; a++) {
            dm[i] += MRT_M[i][a] * (f[a] - E[a]);
            sm[i] += MRT_M[i][a] * S[a];
        }
    }
    double corr[NQ];
    for (int i = 0; i < NQ; i++) {
        double r = mrt_rate(i, tau);
        corr[i] = (-r * dm[i] + (1.0 - 0.5 * r) * sm[i]) / MRT_N2[i];
    }
    for (int a = 0; a < NQ; a++) {
        double v = f[a];
        for (int i = 0; i < NQ; i++) v += MRT_M[i][a] * corr[i];
        out[a] = v;
    }
}

void orc_mrt_basis(double *M) {
    mrt_table();
    for (int i = 0; i < NQ; i++)
        for (int a = 0; a < NQ; a++) M[i * NQ + a] = mrt_row(i, a);
}

/* One MRT collision of 19 populations at a single node (no streaming). */
void orc_collide_node_mrt(const double *f, double rho, const double *u, const double *F, double tau,
                          double *out) {
    double E[NQ], S[NQ];
    for (int a = 0; a < NQ; a++) {
        E[a] = equilibrium(a, rho, u);
        S[a] = source(a, u, F);
    }
    mrt_table();
    mrt_collide(f, E, S, tau, out);
}

static double fplus(const orc_t *o, double phi) { return 0.5 * (1.0 + tanh(phi / o->delta)); }
static double fminus(const orc_t *o, double phi) { return 0.5 * (1.0 - tanh(phi / o->delta)); }

/* feedback modulation of the modulated-feedback equation: m = f+ (polymer in A),
 * f- (polymer in B), 1 (single phase), 0 (no feedback). */
static double modulation(const orc_t *o, double phi) {
    switch (o->phase) {
    case ORC_PHASE_A: return fplus(o, phi);
    case ORC_PHASE_B: return fminus(o, phi);
    case ORC_PHASE_ALL: return 1.0;
    default: return 0.0;
    }
}

/* FENE-P factor f(r) = (L^2 - 3)/(L^2 - tr C).  Returns 0 and sets *bad when tr C >= L^2. */
static double peterlin(const orc_t *o, const double c6[6], int *bad) {
    double tr = c6[0] + c6[1] + c6[2];
    if (!(tr < o->L2)) { *bad |= ORC_F_EXTENSIBILITY; return 0.0; }
    return (o->L2 - 3.0) / (o->L2 - tr);
}

/* C at (x, y, z) with linear-extrapolation ghosts at y = -1 and y = ny. */
static void C_at(const orc_t *o, const double *C, int x, int y, int z, double out[6]) {
    long N = o->N;
    if (y >= 0 && y < o->ny) {
        long n = IDX(o, x, y, z);
        for (int k = 0; k < 6; k++) out[k] = C[k * N + n];
    } else if (y < 0) {
        long n0 = IDX(o, x, 0, z), n1 = IDX(o, x, 1, z);
        for (int k = 0; k < 6; k++) out[k] = 2.0 * C[k * N + n0] - C[k * N + n1];
    } else {
        long n0 = IDX(o, x, o->ny - 1, z), n1 = IDX(o, x, o->ny - 2, z);
        for (int k = 0; k < 6; k++) out[k] = 2.0 * C[k * N + n0] - C[k * N + n1];
    }
}

/* u at (x, y, z) with ghosts reflected through the wall velocity:
 * u(-1) = 2 u_bottom - u(0), u(ny) = 2 u_top - u(ny-1). */
static void u_at(const orc_t *o, int x, int y, int z, double out[3]) {
    long N = o->N;
    if (y >= 0 && y < o->ny) {
        long n = IDX(o, x, y, z);
        for (int d = 0; d < 3; d++) out[d] = o->u[d * N + n];
    } else if (y < 0) {
        long n0 = IDX(o, x, 0, z);
        for (int d = 0; d < 3; d++) out[d] = 2.0 * o->ub[d] - o->u[d * N + n0];
    } else {
        long n0 = IDX(o, x, o->ny - 1, z);
        for (int d = 0; d < 3; d++) out[d] = 2.0 * o->ut[d] - o->u[d * N + n0];
    }
}

/* ------------------------------------------------------------------ stages */

/* S1: densities per species and total momentum. */
static void s1_moments(orc_t *o) {
    long N = o->N;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < o->nz; z++)
        for (int y = 0; y < o->ny; y++)
            for (int x = 0; x < o->nx; x++) {
                long n = IDX(o, x, y, z);
                double jx = 0, jy = 0, jz = 0;
                for (int s = 0; s < o->nc; s++) {
                    double r = 0;
                    for (int a = 0; a < NQ; a++) {
                        double fa = o->f[((long)s * NQ + a) * N + n];
                        r += fa;
                        jx += CX[a] * fa; jy += CY[a] * fa; jz += CZ[a] * fa;
                    }
                    o->rho[(long)s * N + n] = r;
                }
                o->j[n] = jx; o->j[N + n] = jy; o->j[2 * N + n] = jz;
            }
}

/* S2: order parameter.  A single component is a pure phase (phi = 1). */
static void s2_phase(orc_t *o) {
    long N = o->N;
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; n++) {
        if (o->nc == 1) { o->phi[n] = 1.0; continue; }
        double ra = o->rho[n], rb = o->rho[N + n];
        o->phi[n] = (ra - rb) / (ra + rb);
    }
}

/* S3: Shan-Chen inter-species force.  Neighbours across a y wall take the value of
 * the wall-adjacent node (zero normal gradient, neutral wetting). */
static void s3_shan_chen(orc_t *o) {
    long N = o->N;
    if (o->nc == 1) { memset(o->g, 0, sizeof(double) * 3 * N); return; }
#pragma omp parallel for schedule(static)
    for (int z = 0; z < o->nz; z++)
        for (int y = 0; y < o->ny; y++)
            for (int x = 0; x < o->nx; x++) {
                long n = IDX(o, x, y, z);
                for (int s = 0; s < 2; s++) {
                    int so = 1 - s;
                    double acc[3] = {0, 0, 0};
                    for (int a = 1; a < NQ; a++) {
                        int xn = wrap(x + CX[a], o->nx), yn = clampy(o, y + CY[a]), zn = wrap(z + CZ[a], o->nz);
                        double r = o->rho[(long)so * N + IDX(o, xn, yn, zn)];
                        acc[0] += W(a) * r * CX[a];
                        acc[1] += W(a) * r * CY[a];
                        acc[2] += W(a) * r * CZ[a];
                    }
                    double pre = -o->G * o->rho[(long)s * N + n];
                    for (int d = 0; d < 3; d++) o->g[((long)s * 3 + d) * N + n] = pre * acc[d];
                }
            }
}

/* polymer stress at one (possibly ghost) node */
static void stress_at(const orc_t *o, int x, int y, int z, double T[6], int *bad) {
    double c6[6];
    C_at(o, o->C, x, y, z, c6);
    double phi = o->phi[IDX(o, x, clampy(o, y), z)];
    double m = modulation(o, phi);
    double fr = peterlin(o, c6, bad);
    double pre = o->eta_p / o->tau_p * m;
    for (int k = 0; k < 6; k++) T[k] = pre * (fr * c6[k] - (k < 3 ? 1.0 : 0.0));
}

/* S4: divergence of the polymer stress by second-order central differences. */
static void s4_polymer_force(orc_t *o) {
    long N = o->N;
    int bad_all = 0;
#pragma omp parallel for schedule(static) reduction(| : bad_all)
    for (int z = 0; z < o->nz; z++)
        for (int y = 0; y < o->ny; y++)
            for (int x = 0; x < o->nx; x++) {
                long n = IDX(o, x, y, z);
                double div[3] = {0, 0, 0};
                int bad = 0;
                for (int i = 0; i < 3; i++) {
                    int e[3] = {0, 0, 0};
                    e[i] = 1;
                    double Tp[6], Tm[6];
                    stress_at(o, wrap(x + e[0], o->nx), y + e[1], wrap(z + e[2], o->nz), Tp, &bad);
                    stress_at(o, wrap(x - e[0], o->nx), y - e[1], wrap(z - e[2], o->nz), Tm, &bad);
                    for (int jd = 0; jd < 3; jd++) div[jd] += 0.5 * (Tp[sym(i, jd)] - Tm[sym(i, jd)]);
                }
                for (int d = 0; d < 3; d++) o->Fp[d * N + n] = div[d];
                bad_all |= bad;
            }
    o->flags |= bad_all;
}

/* S5 + S6: per-species force and the half-force-corrected barycentric velocity. */
static void s5_s6_force_velocity(orc_t *o) {
    long N = o->N;
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; n++) {
        double rho = 0;
        for (int s = 0; s < o->nc; s++) rho += o->rho[(long)s * N + n];
        double Ft[3] = {0, 0, 0};
        for (int s = 0; s < o->nc; s++) {
            double share = o->coupling == ORC_COUPLING_FORCE ? o->rho[(long)s * N + n] / rho : 0.0;
            for (int d = 0; d < 3; d++) {
                double Fs = o->g[((long)s * 3 + d) * N + n] + share * o->Fp[d * N + n];
                o->F[((long)s * 3 + d) * N + n] = Fs;
                Ft[d] += Fs;
            }
        }
        for (int d = 0; d < 3; d++) o->u[d * N + n] = (o->j[d * N + n] + 0.5 * Ft[d]) / rho;
    }
}

/* S7: local relaxation time interpolated with f+(phi). */
static void s7_tau(orc_t *o) {
    long N = o->N;
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; n++)
        o->tau[n] = (o->nc == 1) ? o->tauA : o->tauB + (o->tauA - o->tauB) * fplus(o, o->phi[n]);
}

/* S8 + S9: BGK collision with source, then push streaming with half-way bounce-back. */
static void s8_s9_collide_stream(orc_t *o) {
    long N = o->N;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < o->nz; z++)
        for (int y = 0; y < o->ny; y++)
            for (int x = 0; x < o->nx; x++) {
                long n = IDX(o, x, y, z);
                double u[3] = {o->u[n], o->u[N + n], o->u[2 * N + n]};
                double tau = o->tau[n];
                double T[6] = {0, 0, 0, 0, 0, 0}, rho = 0.0;
                if (o->coupling == ORC_COUPLING_STRESS) {
                    int bad = 0;
                    stress_at(o, x, y, z, T, &bad);
                    for (int s = 0; s < o->nc; s++) rho += o->rho[(long)s * N + n];
                }
                for (int s = 0; s < o->nc; s++) {
                    double rs = o->rho[(long)s * N + n];
                    double F[3] = {o->F[((long)s * 3) * N + n], o->F[((long)s * 3 + 1) * N + n],
                                   o->F[((long)s * 3 + 2) * N + n]};
                    double Ts[6];
                    for (int k = 0; k < 6; k++) Ts[k] = o->coupling == ORC_COUPLING_STRESS ? rs / rho * T[k] : 0.0;
                    double fm[NQ], Em[NQ], Sm[NQ], pm[NQ];
                    if (o->collision == ORC_COLLISION_MRT) {
                        for (int a = 0; a < NQ; a++) {
                            fm[a] = o->f[((long)s * NQ + a) * N + n];
                            Em[a] = equilibrium(a, rs, u) + equilibrium_stress_term(a, Ts);
                            Sm[a] = source(a, u, F);
                        }
                        mrt_collide(fm, Em, Sm, tau, pm);
                    }
                    for (int a = 0; a < NQ; a++) {
                        double fa = o->f[((long)s * NQ + a) * N + n];
                        double Ea = equilibrium(a, rs, u) + equilibrium_stress_term(a, Ts);
                        double post = o->collision == ORC_COLLISION_MRT
                                          ? pm[a]
                                          : fa - (fa - Ea) / tau + (1.0 - 0.5 / tau) * source(a, u, F);
                        int yd = y + CY[a];
                        if (yd >= 0 && yd < o->ny) {
                            long nd = IDX(o, wrap(x + CX[a], o->nx), yd, wrap(z + CZ[a], o->nz));
                            o->fn[((long)s * NQ + a) * N + nd] = post;
                        } else {
                            const double *uw = yd < 0 ? o->ub : o->ut;
                            double cuw = CX[a] * uw[0] + CY[a] * uw[1] + CZ[a] * uw[2];
                            o->fn[((long)s * NQ + OPP[a]) * N + n] = post - 6.0 * W(a) * rs * cuw;
                        }
                    }
                }
            }
}

/* One step of the Cholesky scheme at one node.  C is the conformation tensor and RC its
 * rate dC/dt (xx, yy, zz, xy, xz, yz order).  With sigma = f C and f = (L^2-3)/(L^2-tr C),
 * f is also (L^2 - 3 + tr sigma)/L^2 and the rate of sigma is f RC + C f^2 tr(RC)/(L^2-3).
 * For sigma = L L^t with L lower triangular, L' = L Phi(A), A = L^-1 sigma' L^-t, Phi(A) the
 * strict lower part of A plus half its diagonal; so (ln l_ii)' = A_ii/2.  The variables
 * y = (ln l11, l21, ln l22, l31, l32, ln l33) take one Adams-Bashforth-2 step with rate ydot
 * and previous rate yprev (forward Euler when hist is 0).  Returns 0, or a fault flag when
 * sigma is not positive definite or a value is not finite. */
static int cholesky_ab2(double L2, const double c[6], const double RC[6], const double *yprev, int hist,
                        double cnew[6], double ydot[6]) {
    double Cm[3][3], Rm[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            Cm[a][b] = c[sym(a, b)];
            Rm[a][b] = RC[sym(a, b)];
        }
    double trC = Cm[0][0] + Cm[1][1] + Cm[2][2], trR = Rm[0][0] + Rm[1][1] + Rm[2][2];
    if (!(trC < L2)) return ORC_F_EXTENSIBILITY;
    double f = (L2 - 3.0) / (L2 - trC);
    double S[3][3], RS[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            S[a][b] = f * Cm[a][b];
            RS[a][b] = f * Rm[a][b] + Cm[a][b] * f * f * trR / (L2 - 3.0);
        }
    /* Cholesky factor of sigma */
    double Lm[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int i = 0; i < 3; i++)
        for (int j = 0; j <= i; j++) {
            double acc = S[i][j];
            for (int k = 0; k < j; k++) acc -= Lm[i][k] * Lm[j][k];
            if (i == j) {
                if (!(acc > 0.0)) return ORC_F_NOT_SPD;
                Lm[i][i] = sqrt(acc);
            } else {
                Lm[i][j] = acc / Lm[j][j];
            }
        }
    /* A = L^-1 RS L^-t: X = L^-1 RS column by column, then A = (L^-1 X^t)^t */
    double X[3][3], A[3][3];
    for (int col = 0; col < 3; col++)
        for (int i = 0; i < 3; i++) {
            double acc = RS[i][col];
            for (int k = 0; k < i; k++) acc -= Lm[i][k] * X[k][col];
            X[i][col] = acc / Lm[i][i];
        }
    for (int col = 0; col < 3; col++)
        for (int i = 0; i < 3; i++) {
            double acc = X[col][i];
            for (int k = 0; k < i; k++) acc -= Lm[i][k] * A[col][k];
            A[col][i] = acc / Lm[i][i];
        }
    double Phi[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int i = 0; i < 3; i++)
        for (int j = 0; j <= i; j++) Phi[i][j] = i == j ? 0.5 * A[i][i] : A[i][j];
    double Ld[3][3];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            Ld[i][j] = 0.0;
            for (int k = 0; k < 3; k++) Ld[i][j] += Lm[i][k] * Phi[k][j];
        }
    ydot[0] = 0.5 * A[0][0];
    ydot[1] = Ld[1][0];
    ydot[2] = 0.5 * A[1][1];
    ydot[3] = Ld[2][0];
    ydot[4] = Ld[2][1];
    ydot[5] = 0.5 * A[2][2];
    double y[6] = {log(Lm[0][0]), Lm[1][0], log(Lm[1][1]), Lm[2][0], Lm[2][1], log(Lm[2][2])};
    for (int k = 0; k < 6; k++) y[k] += hist ? 1.5 * ydot[k] - 0.5 * yprev[k] : ydot[k];
    double Ln[3][3] = {{exp(y[0]), 0, 0}, {y[1], exp(y[2]), 0}, {y[3], y[4], exp(y[5])}};
    double Sn[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            Sn[a][b] = 0.0;
            for (int k = 0; k < 3; k++) Sn[a][b] += Ln[a][k] * Ln[b][k];
        }
    double fn = (L2 - 3.0 + Sn[0][0] + Sn[1][1] + Sn[2][2]) / L2;
    for (int a = 0; a < 3; a++)
        for (int b = a; b < 3; b++) cnew[sym(a, b)] = Sn[a][b] / fn;
    for (int k = 0; k < 6; k++)
        if (!isfinite(cnew[k]) || !isfinite(ydot[k])) return ORC_F_NONFINITE;
    return 0;
}

void orc_cholesky_ab2(double L2, const double *c, const double *RC, const double *yprev, int hist,
                      double *cnew, double *ydot, int *flag) {
    *flag = cholesky_ab2(L2, c, RC, yprev, hist, cnew, ydot);
}

/* S10: explicit Euler FENE-P update with upwind advection and central velocity
 * gradients, dt = 1 lattice step (or the Cholesky scheme, see cholesky_ab2). */
static void s10_fenep(orc_t *o) {
    long N = o->N;
    int bad_all = 0;
#pragma omp parallel for schedule(static) reduction(| : bad_all)
    for (int z = 0; z < o->nz; z++)
        for (int y = 0; y < o->ny; y++)
            for (int x = 0; x < o->nx; x++) {
                long n = IDX(o, x, y, z);
                int bad = 0;
                double c0[6];
                C_at(o, o->C, x, y, z, c0);
                double u0[3] = {o->u[n], o->u[N + n], o->u[2 * N + n]};
                /* velocity gradient G[i][j] = d_i u_j */
                double Gm[3][3];
                double adv[6] = {0, 0, 0, 0, 0, 0};
                for (int i = 0; i < 3; i++) {
                    int e[3] = {0, 0, 0};
                    e[i] = 1;
                    int xp = wrap(x + e[0], o->nx), yp = y + e[1], zp = wrap(z + e[2], o->nz);
                    int xm = wrap(x - e[0], o->nx), ym = y - e[1], zm = wrap(z - e[2], o->nz);
                    double up[3], um[3];
                    u_at(o, xp, yp, zp, up);
                    u_at(o, xm, ym, zm, um);
                    for (int jd = 0; jd < 3; jd++) Gm[i][jd] = 0.5 * (up[jd] - um[jd]);
                    double cn[6];
                    if (o->fene == ORC_FENE_CHOLESKY_AB2) {
                        /* second-order central difference, and the artificial diffusivity */
                        double cp[6];
                        C_at(o, o->C, xp, yp, zp, cp);
                        C_at(o, o->C, xm, ym, zm, cn);
                        for (int k = 0; k < 6; k++)
                            adv[k] += u0[i] * 0.5 * (cp[k] - cn[k]) - o->kappa * (cp[k] - 2.0 * c0[k] + cn[k]);
                    } else if (u0[i] >= 0.0) {
                        /* first-order upwind difference along i */
                        C_at(o, o->C, xm, ym, zm, cn);
                        for (int k = 0; k < 6; k++) adv[k] += u0[i] * (c0[k] - cn[k]);
                    } else {
                        C_at(o, o->C, xp, yp, zp, cn);
                        for (int k = 0; k < 6; k++) adv[k] += u0[i] * (cn[k] - c0[k]);
                    }
                }
                double fr = peterlin(o, c0, &bad);
                double Cm[3][3];
                for (int a = 0; a < 3; a++)
                    for (int b = 0; b < 3; b++) Cm[a][b] = c0[sym(a, b)];
                double RC[6];
                for (int a = 0; a < 3; a++)
                    for (int b = a; b < 3; b++) {
                        double stretch = 0;
                        for (int k = 0; k < 3; k++) stretch += Gm[k][a] * Cm[k][b] + Cm[a][k] * Gm[k][b];
                        int kk = sym(a, b);
                        double relax = (fr * c0[kk] - (a == b ? 1.0 : 0.0)) / o->tau_p;
                        RC[kk] = -adv[kk] + stretch - relax;
                    }
                if (o->fene == ORC_FENE_CHOLESKY_AB2) {
                    double yp6[6], cn6[6], yd6[6];
                    for (int k = 0; k < 6; k++) yp6[k] = o->Hp[k * N + n];
                    bad |= cholesky_ab2(o->L2, c0, RC, yp6, o->have_hist, cn6, yd6);
                    for (int k = 0; k < 6; k++) {
                        o->Cn[k * N + n] = cn6[k];
                        o->Hn[k * N + n] = yd6[k];
                    }
                } else {
                    for (int k = 0; k < 6; k++) o->Cn[k * N + n] = c0[k] + RC[k];
                }
                bad_all |= bad;
            }
    o->flags |= bad_all;
}

/* S11: fault checks on the new state (non-finite, extensibility, leading minors). */
static void s11_checks(orc_t *o) {
    long N = o->N;
    int bad_all = 0;
#pragma omp parallel for schedule(static) reduction(| : bad_all)
    for (long n = 0; n < N; n++) {
        int bad = 0;
        for (int s = 0; s < o->nc; s++)
            for (int a = 0; a < NQ; a++)
                if (!isfinite(o->fn[((long)s * NQ + a) * N + n])) bad |= ORC_F_NONFINITE;
        double c[6];
        for (int k = 0; k < 6; k++) {
            c[k] = o->Cn[k * N + n];
            if (!isfinite(c[k])) bad |= ORC_F_NONFINITE;
        }
        if (!(c[0] + c[1] + c[2] < o->L2)) bad |= ORC_F_EXTENSIBILITY;
        double m1 = c[0];
        double m2 = c[0] * c[1] - c[3] * c[3];
        double m3 = c[0] * (c[1] * c[2] - c[5] * c[5]) - c[3] * (c[3] * c[2] - c[5] * c[4]) +
                    c[4] * (c[3] * c[5] - c[1] * c[4]);
        if (!(m1 > 0 && m2 > 0 && m3 > 0)) bad |= ORC_F_NOT_SPD;
        bad_all |= bad;
    }
    o->flags |= bad_all;
}

/* S1..S6 on the current state: fills rho, j, phi, g, Fp, F, u. */
static void derived_fields(orc_t *o) {
    s1_moments(o);
    s2_phase(o);
    s3_shan_chen(o);
    s4_polymer_force(o);
    s5_s6_force_velocity(o);
}

/* ------------------------------------------------------------------ API */

/* f = E(rho_s, u) (no non-equilibrium part) and C as given.  rho: [nc][N], u: [3][N],
 * C: [6][N] in (xx, yy, zz, xy, xz, yz) order. */
int orc_set_fields(orc_t *o, const double *rho, const double *u, const double *C) {
    long N = o->N;
    for (long n = 0; n < N; n++) {
        double un[3] = {u[n], u[N + n], u[2 * N + n]};
        for (int s = 0; s < o->nc; s++)
            for (int a = 0; a < NQ; a++)
                o->f[((long)s * NQ + a) * N + n] = equilibrium(a, rho[(long)s * N + n], un);
    }
    memcpy(o->C, C, sizeof(double) * 6 * N);
    o->steps = 0;
    o->flags = 0;
    o->have_hist = 0;
    return 0;
}

/* Advance nsteps; stops after the first step that raises a fault flag and returns the flags. */
int orc_step(orc_t *o, long nsteps) {
    for (long t = 0; t < nsteps; t++) {
        o->flags = 0;
        derived_fields(o);
        s7_tau(o);
        s8_s9_collide_stream(o);
        s10_fenep(o);
        s11_checks(o);
        double *tmp = o->f; o->f = o->fn; o->fn = tmp;
        tmp = o->C; o->C = o->Cn; o->Cn = tmp;
        if (o->fene == ORC_FENE_CHOLESKY_AB2) {
            tmp = o->Hp; o->Hp = o->Hn; o->Hn = tmp;
            o->have_hist = 1;
        }
        o->steps++;
        if (o->flags) return o->flags;
    }
    return 0;
}

/* Macroscopic fields of the current state; u includes the half-force shift.
 * Any pointer may be NULL. */
void orc_get_fields(orc_t *o, double *rho, double *u, double *C) {
    long N = o->N;
    int saved = o->flags;
    derived_fields(o);
    o->flags = saved;
    if (rho) memcpy(rho, o->rho, sizeof(double) * o->nc * N);
    if (u) memcpy(u, o->u, sizeof(double) * 3 * N);
    if (C) memcpy(C, o->C, sizeof(double) * 6 * N);
}

/* Intermediate force fields of the current state (for tests): g [nc][3][N], Fp [3][N],
 * F [nc][3][N].  Any pointer may be NULL. */
void orc_get_forces(orc_t *o, double *g, double *Fp, double *F) {
    long N = o->N;
    int saved = o->flags;
    derived_fields(o);
    o->flags = saved;
    if (g) memcpy(g, o->g, sizeof(double) * o->nc * 3 * N);
    if (Fp) memcpy(Fp, o->Fp, sizeof(double) * 3 * N);
    if (F) memcpy(F, o->F, sizeof(double) * o->nc * 3 * N);
}

void orc_get_pops(const orc_t *o, double *f) { memcpy(f, o->f, sizeof(double) * o->nc * NQ * o->N); }

/* Diagnostics record (all FP64, serial fixed-order sums):
 *  [0..1] mass per species, [2..4] total momentum sum rho u, [5] W = sum w with
 *  w = max(phi, 0), [6..8] centroid, [9..14] second moments about the centroid
 *  (xx, yy, zz, xy, xz, yz) divided by W, [15] D, [16] theta in degrees,
 *  [17] min(L^2 - tr C), [18] min leading minor of C, [19] max |u|, [20] flags,
 *  [21] mean of tr C - 3 over the polymer phase weighted by the feedback modulation.
 * D = (a - b)/(a + b) and theta = angle of the major axis with x, from the x-y block
 * of the second-moment tensor (Sec. 4, deformation parameter and orientation). */
void orc_diagnostics(orc_t *o, double *out) {
    long N = o->N;
    int saved = o->flags;
    derived_fields(o);
    o->flags = saved;
    for (int k = 0; k < 22; k++) out[k] = 0.0;
    double mass[2] = {0, 0}, mom[3] = {0, 0, 0};
    double Wt = 0, sx = 0, sy = 0, sz = 0;
    double minL = INFINITY, minM = INFINITY, maxu = 0, pex = 0, pw = 0;
    for (int z = 0; z < o->nz; z++)
        for (int y = 0; y < o->ny; y++)
            for (int x = 0; x < o->nx; x++) {
                long n = IDX(o, x, y, z);
                double rho = 0;
                for (int s = 0; s < o->nc; s++) { mass[s] += o->rho[(long)s * N + n]; rho += o->rho[(long)s * N + n]; }
                double un[3] = {o->u[n], o->u[N + n], o->u[2 * N + n]};
                for (int d = 0; d < 3; d++) mom[d] += rho * un[d];
                double um = sqrt(un[0] * un[0] + un[1] * un[1] + un[2] * un[2]);
                if (um > maxu) maxu = um;
                double w = o->phi[n] > 0 ? o->phi[n] : 0.0;
                Wt += w; sx += w * x; sy += w * y; sz += w * z;
                double c[6];
                for (int k = 0; k < 6; k++) c[k] = o->C[k * N + n];
                double mp = modulation(o, o->phi[n]);
                pex += mp * (c[0] + c[1] + c[2] - 3.0);
                pw += mp;
                double l = o->L2 - (c[0] + c[1] + c[2]);
                if (l < minL) minL = l;
                double m1 = c[0], m2 = c[0] * c[1] - c[3] * c[3];
                double m3 = c[0] * (c[1] * c[2] - c[5] * c[5]) - c[3] * (c[3] * c[2] - c[5] * c[4]) +
                            c[4] * (c[3] * c[5] - c[1] * c[4]);
                double mm = m1 < m2 ? m1 : m2;
                mm = mm < m3 ? mm : m3;
                if (mm < minM) minM = mm;
            }
    double xc = sx / Wt, yc = sy / Wt, zc = sz / Wt;
    double M[6] = {0, 0, 0, 0, 0, 0};
    for (int z = 0; z < o->nz; z++)
        for (int y = 0; y < o->ny; y++)
            for (int x = 0; x < o->nx; x++) {
                long n = IDX(o, x, y, z);
                double w = o->phi[n] > 0 ? o->phi[n] : 0.0;
                double dx = x - xc, dy = y - yc, dz = z - zc;
                M[0] += w * dx * dx; M[1] += w * dy * dy; M[2] += w * dz * dz;
                M[3] += w * dx * dy; M[4] += w * dx * dz; M[5] += w * dy * dz;
            }
    for (int k = 0; k < 6; k++) M[k] /= Wt;
    /* eigenvalues of the x-y block */
    double tr = M[0] + M[1], df = M[0] - M[1];
    double rad = sqrt(0.25 * df * df + M[3] * M[3]);
    double l1 = 0.5 * tr + rad, l2 = 0.5 * tr - rad;
    if (l2 < 0) l2 = 0;
    double a = sqrt(l1), b = sqrt(l2);
    double D = (a + b) > 0 ? (a - b) / (a + b) : 0.0;
    double theta = (rad > 0) ? 0.5 * atan2(2.0 * M[3], df) * 180.0 / 3.14159265358979323846 : 0.0;
    out[0] = mass[0]; out[1] = mass[1];
    out[2] = mom[0]; out[3] = mom[1]; out[4] = mom[2];
    out[5] = Wt; out[6] = xc; out[7] = yc; out[8] = zc;
    for (int k = 0; k < 6; k++) out[9 + k] = M[k];
    out[15] = D; out[16] = theta; out[17] = minL; out[18] = minM; out[19] = maxu;
    out[20] = (double)o->flags;
    out[21] = pw > 0 ? pex / pw : 0.0;
}

/* ---------------------------------------------------------- helpers for pins */

void orc_lattice(int *c, double *w, int *opp) {
    for (int a = 0; a < NQ; a++) {
        c[3 * a] = CX[a]; c[3 * a + 1] = CY[a]; c[3 * a + 2] = CZ[a];
        w[a] = W(a);
        opp[a] = OPP[a];
    }
}

void orc_equilibrium(double rho, const double *u, double *E) {
    for (int a = 0; a < NQ; a++) E[a] = equilibrium(a, rho, u);
}

/* Equilibrium with the polymer stress T_s in its second moment (single node). */
void orc_equilibrium_stress(double rho, const double *u, const double *Ts, double *E) {
    for (int a = 0; a < NQ; a++) E[a] = equilibrium(a, rho, u) + equilibrium_stress_term(a, Ts);
}

void orc_source(const double *u, const double *F, double *S) {
    for (int a = 0; a < NQ; a++) S[a] = source(a, u, F);
}

/* One BGK collision of 19 populations at a single node (no streaming). */
void orc_collide_node(const double *f, double rho, const double *u, const double *F, double tau,
                      double *out) {
    for (int a = 0; a < NQ; a++)
        out[a] = f[a] - (f[a] - equilibrium(a, rho, u)) / tau + (1.0 - 0.5 / tau) * source(a, u, F);
}

/* Prescribed-velocity ("kinematic") FENE-P stepping: the LB part is not run, u is the
 * given field [3][N] (held fixed), and only S10 is applied nsteps times.  Used by the
 * rheology pins (the paper's homogeneous benchmarks switch the feedback off). */
int orc_fenep_kinematic(orc_t *o, const double *u, long nsteps) {
    long N = o->N;
    memcpy(o->u, u, sizeof(double) * 3 * N);
    for (long t = 0; t < nsteps; t++) {
        o->flags = 0;
        s10_fenep(o);
        double *tmp = o->C; o->C = o->Cn; o->Cn = tmp;
        if (o->fene == ORC_FENE_CHOLESKY_AB2) {
            tmp = o->Hp; o->Hp = o->Hn; o->Hn = tmp;
            o->have_hist = 1;
        }
        if (o->flags) return o->flags;
    }
    return 0;
}

void orc_get_C(const orc_t *o, double *C) { memcpy(C, o->C, sizeof(double) * 6 * o->N); }
void orc_set_C(orc_t *o, const double *C) { memcpy(o->C, C, sizeof(double) * 6 * o->N); }

#ifdef _OPENMP
#include <omp.h>
int orc_threads(void) { return omp_get_max_threads(); }
/* threads of the following parallel regions (results do not depend on it) */
void orc_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
#else
int orc_threads(void) { return 1; }
void orc_set_threads(int n) { (void)n; }
#endif
