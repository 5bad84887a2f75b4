/*
 * cg_oracle.c -- plain FP64 CPU oracle of the colour-gradient LBM step.
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU baseline
 * of the benchmark load this file's library.  It shares nothing with the HIP
 * implementation.
 *
 * Source: Douillet-Grellier, Leclaire, Vidal, Bertrand, De Vuyst,
 * "Comparison of multiphase SPH and LBM approaches for the simulation of
 * intermittent flows", arXiv:1903.01168.  Section numbers below refer to it.
 *
 * Each time step is done as separate full-lattice passes, in the order of the
 * operator splitting of Section 2 (collision, perturbation, recolouring,
 * streaming), written as a "pull": the populations stored after the previous
 * recolouring are streamed first, then the three collision sub-operators act.
 *
 * Readings of passages that are silent, garbled or inconsistent (each one is
 * listed in the design notes of the repository):
 *  R1  velocity numbering: the one implied by the rows of M in Appendix B
 *      (rows 3 and 5 are c_x and c_y): 1..4 axis, 5..8 diagonal.  W_i, phi_i,
 *      B_i and xi_i are taken by the class |c_i|^2 (0, 1, 2).
 *  R2  alpha of the heavier fluid from equal reference pressures
 *      rho0_r (1-alpha_r) = rho0_b (1-alpha_b); alpha of the lighter one given.
 *  R3  colour field psi = +1 in pure red (as the formula of Sec. 2.1.1 reads).
 *  R4  body force: Guo forcing on the colour-blind populations, with the
 *      half-force velocity shift in the equilibrium (no scheme in the paper).
 *  R5  perturbation: the colour-blind sum of the two A/2 terms, i.e. A|F|[..];
 *      skipped (with the recolouring term) when |F| <= 1e-12.
 *  R6  walls: halfway (link) bounce-back; psi on wall ghost nodes is the
 *      W-weighted mean of psi over fluid neighbours (Sec. 2.4, without the
 *      stray c_i factor); open-boundary ghost columns copy the nearest column.
 *  R7  open boundaries (Sec. 2.5): Zou-He formulas rotated to a west velocity
 *      inlet and an east pressure outlet; inlet colour prescribed per row;
 *      outlet colour = volume fraction of the six populations that stream in
 *      from the domain, clamped to [0, 1] as the (phi + 1) / 2 of a colour
 *      field in [-1, 1]; outlet densities rho_k = chi_k p_out / c_s,k^2.
 *  R8  collision is colour-blind (same omega_eff and S for both colours); the
 *      percolor switch runs the per-colour form for comparison.
 *  R6b free slip (Sec. 2.5 item 1): a diagonal population that would come
 *      from beyond the wall is the mirrored one that left the upstream node of
 *      the same row; the wall-normal one bounces back.
 *  R11 contact angle (Sec. 2.4): theta is the red fluid's angle, measured
 *      through red; the gradient (into red) is turned to pi - theta from the
 *      wall normal; at theta = 0 or pi the two candidates are one vector.
 *  R12 Hermite equilibrium (Sec. 2.1.3): the garbled factor (3 c_i - 4) read
 *      as (3 |c_i|^2 - 4).
 *  R13 Navier-Stokes source (Sec. 2.1.3): C_7 = (1 - s_7/2)(dQx/dx - dQy/dy)
 *      (printed with a factor 3, omega_eff and a plus sign).
 *  R14 Q^k = (1.8 alpha_k - 0.8) rho_k u with the half-force velocity; its
 *      ghost values beyond walls and open faces follow the colour field's
 *      rules (R6) (the paper gives no rule).  Zou-He H uses the prescribed (inlet) or
 *      measured (outlet) colour fractions of R7.
 *  R15 the more isotropic gradient the paper mentions (Sec. 4) as an option:
 *      the 25-point second-neighbour stencil isotropic to 8th order.  Its
 *      outer ghost cells: beyond an open face the nearest column (R6);
 *      beyond a wall the inner ghost row (Sec. 2.4 defines solid nodes with
 *      fluid neighbours only); corner cells beyond both take the inner ghost
 *      column of the ghost row.
 *  R6, R14 and R15's ghost values are pinned by closed-form gradients of
 *  fields that vary along the wall; where the paper leaves a rule open (R7's
 *  outlet colour, R14's Q beyond a wall, R15's outer ghost row) the
 *  alternative reading is selectable (or_params.alt) so that its effect can
 *  be measured.
 */
#include "cg_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Lattice (Sec. 2, R1)                                                */
/* ------------------------------------------------------------------ */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

static int cls(int i) { return CX[i] * CX[i] + CY[i] * CY[i]; }

static const double PI_ = 3.14159265358979323846;

static int opposite(int i)
{
    for (int j = 0; j < 9; ++j)
        if (CX[j] == -CX[i] && CY[j] == -CY[i]) return j;
    return -1;
}

/* the direction with the same c_x and the opposite c_y */
static int mirror_y(int i)
{
    for (int j = 0; j < 9; ++j)
        if (CX[j] == CX[i] && CY[j] == -CY[i]) return j;
    return i;
}

/* D2Q9 weights, Sec. 2.1.1 */
static double Wt(int i)
{
    static const double w[3] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 36.0};
    return w[cls(i)];
}

/* phi^k_i of the density-ratio equilibrium, Sec. 2.1.1 */
static double phi(int i, double alpha)
{
    switch (cls(i)) {
    case 0: return alpha;
    case 1: return (1.0 - alpha) / 5.0;
    default: return (1.0 - alpha) / 20.0;
    }
}

/* B_i of the perturbation operator, Sec. 2.2 */
static double Bcoef(int i)
{
    static const double b[3] = {-4.0 / 27.0, 2.0 / 27.0, 5.0 / 108.0};
    return b[cls(i)];
}

/* xi_i of the S2I4 gradient, Sec. 2.2 eq. (colorGradient) */
static double xi(int i)
{
    static const double x[3] = {0.0, 1.0 / 3.0, 1.0 / 12.0};
    return x[cls(i)];
}

void or_lattice(int *cx, int *cy, int *opp, double *W)
{
    for (int i = 0; i < 9; ++i) {
        cx[i] = CX[i];
        cy[i] = CY[i];
        opp[i] = opposite(i);
        W[i] = Wt(i);
    }
}

void or_tables(double alpha, double *ph, double *B, double *x)
{
    for (int i = 0; i < 9; ++i) {
        ph[i] = phi(i, alpha);
        B[i] = Bcoef(i);
        x[i] = xi(i);
    }
}

/* Sec. 2.1.1 eq. (gammaAlphaBeta) read as equal reference pressures (R2) */
void or_alphas(double rho0_r, double rho0_b, double alpha_light, double *alpha_r, double *alpha_b)
{
    if (rho0_r <= rho0_b) {
        *alpha_r = alpha_light;
        *alpha_b = 1.0 - (1.0 - alpha_light) * rho0_r / rho0_b;
    } else {
        *alpha_b = alpha_light;
        *alpha_r = 1.0 - (1.0 - alpha_light) * rho0_b / rho0_r;
    }
}

/* Appendix B, as printed */
static const double MRT_M[81] = {
     1,  1,  1,  1,  1,  1,  1,  1,  1,
    -4, -1, -1, -1, -1,  2,  2,  2,  2,
     4, -2, -2, -2, -2,  1,  1,  1,  1,
     0,  1,  0, -1,  0,  1, -1, -1,  1,
     0, -2,  0,  2,  0,  1, -1, -1,  1,
     0,  0,  1,  0, -1,  1,  1, -1, -1,
     0,  0, -2,  0,  2,  1,  1, -1, -1,
     0,  1, -1,  1, -1,  0,  0,  0,  0,
     0,  0,  0,  0,  0,  1, -1,  1, -1,
};
static const double MRT_MINV36[81] = {
    4, -4,  4,  0,  0,  0,  0,  0,  0,
    4, -1, -2,  6, -6,  0,  0,  9,  0,
    4, -1, -2,  0,  0,  6, -6, -9,  0,
    4, -1, -2, -6,  6,  0,  0,  9,  0,
    4, -1, -2,  0,  0, -6,  6, -9,  0,
    4,  2,  1,  6,  3,  6,  3,  0,  9,
    4,  2,  1, -6, -3,  6,  3,  0, -9,
    4,  2,  1, -6, -3, -6, -3,  0,  9,
    4,  2,  1,  6,  3, -6, -3,  0, -9,
};

/* Sec. 2.1.1 eq. (equilibrium) */
void or_equilibrium(double rho_k, double ux, double uy, double alpha_k, double *out9)
{
    double uu = ux * ux + uy * uy;
    for (int i = 0; i < 9; ++i) {
        double cu = CX[i] * ux + CY[i] * uy;
        out9[i] = rho_k * (phi(i, alpha_k) + Wt(i) * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
    }
}

/* Sec. 2.1.3 eq. (equilibrium_hermite): the linear term carries the factor
 * 1 + (3 c_s^2 - 1)(3 |c_i|^2 - 4) / 2 (R12: |c_i|^2 for the garbled c_i;
 * with it the equilibrium keeps mass and momentum and its third moments
 * sum c_x^2 c_y, sum c_x c_y^2 become c_s^2 rho u_y, c_s^2 rho u_x). */
void or_equilibrium_hermite(double rho_k, double ux, double uy, double alpha_k, double *out9)
{
    double uu = ux * ux + uy * uy;
    double k3 = 3.0 * (3.0 * (1.0 - alpha_k) / 5.0) - 1.0;     /* 3 c_s^2 - 1 */
    for (int i = 0; i < 9; ++i) {
        double cu = CX[i] * ux + CY[i] * uy;
        double lin = 3.0 * cu * (1.0 + 0.5 * k3 * (3.0 * cls(i) - 4.0));
        out9[i] = rho_k * (phi(i, alpha_k) + Wt(i) * (lin + 4.5 * cu * cu - 1.5 * uu));
    }
}

/* Sec. 2.1.3: the source U = M^{-1} C added to the MRT collision, with
 * C = (0, C_1, 0, 0, 0, 0, 0, C_7, 0), C_1 = 3 (1 - s_1/2) (dQx/dx + dQy/dy)
 * and (R13) C_7 = (1 - s_7/2) (dQx/dx - dQy/dy): row 1 of M is
 * 3 (c_x^2 + c_y^2) - 4 and row 7 is c_x^2 - c_y^2, and the lattice's
 * remaining third-moment defect sum c_x^3 N^e - 3 c_s^2 rho u_x = Q_x (and
 * likewise in y) enters the momentum flux as diag(dQx/dx, dQy/dy). */
void or_ns_source(double dQxdx, double dQydy, double s1, double s7, double *out9)
{
    double Cm[9] = {0.0};
    Cm[1] = 3.0 * (1.0 - s1 / 2.0) * (dQxdx + dQydy);
    Cm[7] = (1.0 - s7 / 2.0) * (dQxdx - dQydy);
    for (int i = 0; i < 9; ++i) {
        out9[i] = 0.0;
        for (int j = 0; j < 9; ++j) out9[i] += MRT_MINV36[i * 9 + j] / 36.0 * Cm[j];
    }
}

/* Sec. 2.1.1: omega_eff, quadratic interpolation across the interface */
double or_omega_eff(double psi, double omega_r, double omega_b, double delta)
{
    double chi = 2.0 * omega_r * omega_b / (omega_r + omega_b);
    double eta = 2.0 * (omega_r - chi) / delta;
    double kappa = -eta / (2.0 * delta);
    double lam = 2.0 * (chi - omega_b) / delta;
    double nu = lam / (2.0 * delta);
    if (psi > delta) return omega_r;
    if (psi > 0.0) return chi + eta * psi + kappa * psi * psi;
    if (psi >= -delta) return chi + lam * psi + nu * psi * psi;
    return omega_b;
}

/* Sec. 2.2 eq. (colorGradient) on a 3x3 patch */
void or_gradient3x3(const double *psi9, double *F2)
{
    F2[0] = 0.0;
    F2[1] = 0.0;
    for (int i = 1; i < 9; ++i) {
        double v = psi9[(CY[i] + 1) * 3 + (CX[i] + 1)];
        F2[0] += xi(i) * CX[i] * v;
        F2[1] += xi(i) * CY[i] * v;
    }
}

/* Second-neighbour colour gradient (the more isotropic operator the paper
 * points to in Sec. 4 as an option, R15): F = sum over the 24 nodes with
 * |dx|, |dy| <= 2 of w(|c|^2) c psi(x + c), with the weights of the
 * 8th-order isotropic 25-point stencil, w(1) = 4/21, w(2) = 4/45,
 * w(4) = 1/60, w(5) = 2/315, w(8) = 1/5040 (second moment sum w c c = I). */
void or_gradient5x5(const double *psi25, double *F2)
{
    F2[0] = F2[1] = 0.0;
    for (int dy = -2; dy <= 2; ++dy)
        for (int dx = -2; dx <= 2; ++dx) {
            int c2 = dx * dx + dy * dy;
            double w = c2 == 1 ? 4.0 / 21.0 : c2 == 2 ? 4.0 / 45.0 : c2 == 4 ? 1.0 / 60.0
                     : c2 == 5 ? 2.0 / 315.0 : c2 == 8 ? 1.0 / 5040.0 : 0.0;
            F2[0] += w * dx * psi25[(dy + 2) * 5 + (dx + 2)];
            F2[1] += w * dy * psi25[(dy + 2) * 5 + (dx + 2)];
        }
}

/* Sec. 2.4: orientation of the colour gradient at a fluid node next to a
 * wall.  n* = F/|F|; the two unit normals that make the angle theta with
 * the wall normal ns; the one closer to n* (ns itself on a tie); |F| kept.
 * At theta = 0 or pi the two candidates are one vector, which is taken: the
 * tie rule is read as meant for n* halfway between two distinct ones (R11). */
void or_wetting(const double *F2, const double *ns2, double theta, double *out2)
{
    double Fm = sqrt(F2[0] * F2[0] + F2[1] * F2[1]);
    out2[0] = F2[0];
    out2[1] = F2[1];
    if (Fm <= 1e-12) return;                 /* no gradient, nothing to orient (R5) */
    double nx = F2[0] / Fm, ny = F2[1] / Fm;
    double c = cos(theta), s = sin(theta);
    if (fabs(s) <= 1e-15) {                  /* theta = 0 or pi: the two candidates coincide (R11) */
        out2[0] = Fm * c * ns2[0];
        out2[1] = Fm * c * ns2[1];
        return;
    }
    double n1x = ns2[0] * c - ns2[1] * s, n1y = ns2[1] * c + ns2[0] * s;
    double n2x = ns2[0] * c + ns2[1] * s, n2y = ns2[1] * c - ns2[0] * s;
    double D1 = sqrt((nx - n1x) * (nx - n1x) + (ny - n1y) * (ny - n1y));
    double D2 = sqrt((nx - n2x) * (nx - n2x) + (ny - n2y) * (ny - n2y));
    double ox, oy;
    if (D1 < D2) { ox = n1x; oy = n1y; }
    else if (D1 > D2) { ox = n2x; oy = n2y; }
    else { ox = ns2[0]; oy = ns2[1]; }
    out2[0] = Fm * ox;
    out2[1] = Fm * oy;
}

/* Sec. 2.2 eq. (perturbation), colour-blind sum (R5): the term added to N* */
void or_perturbation(const double *F2, double A, double *out9)
{
    double F = sqrt(F2[0] * F2[0] + F2[1] * F2[1]);
    for (int i = 0; i < 9; ++i) {
        if (F <= 1e-12) {
            out9[i] = 0.0;
            continue;
        }
        double Fc = F2[0] * CX[i] + F2[1] * CY[i];
        out9[i] = A * F * (Wt(i) * Fc * Fc / (F * F) - Bcoef(i));
    }
}

/* Sec. 2.3 eq. (recoloringOperator) */
void or_recolor(const double *Nss9, double rho_r, double rho_b, const double *F2, double beta,
                double alpha_r, double alpha_b, double *out_r9, double *out_b9)
{
    double rho = rho_r + rho_b;
    double F = sqrt(F2[0] * F2[0] + F2[1] * F2[1]);
    for (int i = 0; i < 9; ++i) {
        double seg = 0.0;
        if (i != 0 && F > 1e-12) {
            double ci = sqrt((double)cls(i));
            double cosphi = (CX[i] * F2[0] + CY[i] * F2[1]) / (ci * F);
            /* sum over colours of the equilibrium at zero velocity */
            double eq0 = rho_r * phi(i, alpha_r) + rho_b * phi(i, alpha_b);
            seg = beta * rho_r * rho_b / (rho * rho) * cosphi * eq0;
        }
        out_r9[i] = rho_r / rho * Nss9[i] + seg;
        out_b9[i] = rho_b / rho * Nss9[i] - seg;
    }
}

/* Sec. 2.5 item 3, velocity inlet rotated to the west face (R7).
 * Unknowns 1, 5, 8; the non-equilibrium bounce-back closes the system.
 * kap = sum_k chi_k (3 c_s,k^2 - 1) with the Hermite equilibrium of
 * Sec. 2.1.3 (its corrective term H = kap rho v_x / 3), 0 with the plain one. */
double or_zouhe_west(double *N, double vx, double vy, double kap)
{
    double rho = (N[0] + N[2] + N[4] + 2.0 * (N[3] + N[6] + N[7])) / (1.0 - vx);
    double H = kap * rho * vx / 3.0;
    N[1] = N[3] + 2.0 / 3.0 * rho * vx - H;
    N[5] = N[7] - 0.5 * (N[2] - N[4]) + 0.5 * rho * vy + rho * vx / 6.0 + 0.5 * H;
    N[8] = N[6] + 0.5 * (N[2] - N[4]) - 0.5 * rho * vy + rho * vx / 6.0 + 0.5 * H;
    return rho;
}

/* Sec. 2.5 item 3, pressure outlet rotated to the east face (R7); kap as
 * for the inlet. */
double or_zouhe_east(double *N, double rho, double vy, double kap)
{
    double vx = (N[0] + N[2] + N[4] + 2.0 * (N[1] + N[5] + N[8])) / rho - 1.0;
    double H = kap * rho * vx / 3.0;
    N[3] = N[1] - 2.0 / 3.0 * rho * vx + H;
    N[6] = N[8] - 0.5 * (N[2] - N[4]) + 0.5 * rho * vy - rho * vx / 6.0 - 0.5 * H;
    N[7] = N[5] + 0.5 * (N[2] - N[4]) - 0.5 * rho * vy - rho * vx / 6.0 - 0.5 * H;
    return vx;
}

void or_mrt_matrices(double *M81, double *Minv81)
{
    for (int a = 0; a < 81; ++a) {
        M81[a] = MRT_M[a];
        Minv81[a] = MRT_MINV36[a] / 36.0;
    }
}

/* relaxation rates s_j of Sec. 2.1.2 eq. (relax_times) */
static void mrt_rates(double omega, double lambda, double *s)
{
    for (int j = 0; j < 7; ++j) s[j] = lambda * omega;
    s[7] = omega;
    s[8] = omega;
}

/* x -> M^{-1} diag(d) M x */
static void mrt_apply(const double *x, const double *d, double *out)
{
    double m[9];
    for (int j = 0; j < 9; ++j) {
        m[j] = 0.0;
        for (int i = 0; i < 9; ++i) m[j] += MRT_M[j * 9 + i] * x[i];
        m[j] *= d[j];
    }
    for (int i = 0; i < 9; ++i) {
        out[i] = 0.0;
        for (int j = 0; j < 9; ++j) out[i] += MRT_MINV36[i * 9 + j] / 36.0 * m[j];
    }
}

/* Sec. 2.1.2 eq. (singleCollisionMRT) */
void or_mrt_collide(const double *N, const double *Neq, double omega, double lambda, double *out9)
{
    double s[9], d[9], r[9];
    mrt_rates(omega, lambda, s);
    for (int i = 0; i < 9; ++i) d[i] = N[i] - Neq[i];
    mrt_apply(d, s, r);
    for (int i = 0; i < 9; ++i) out9[i] = N[i] - r[i];
}

/* ------------------------------------------------------------------ */
/* Lattice-level driver                                                */
/* ------------------------------------------------------------------ */
struct or_sim {
    or_params p;
    double alpha[2], rho0[2], cs2[2], omega[2];
    double *post;   /* [2][9][ny][nx] post-recolouring state            */
    double *strm;   /* [2][9][ny][nx] streamed + boundary-completed     */
    double *rho;    /* [2][ny][nx] colour densities used by the step    */
    double *ux, *uy;
    double *psi;    /* [ny+4][nx+4] colour field with a ghost layer of two cells */
    double *q;      /* [2 colours][2 components][ny+4][nx+4] Q^k of Sec. 2.1.3, same layout */
    signed char *inlet_color;
    long step;
};

#define POP(a, k, i, y, x) ((a)[((((size_t)(k) * 9 + (i)) * ny + (y)) * nx) + (x)])

static int wrap(int v, int n) { return ((v % n) + n) % n; }

/* fields with ghost cells: two cells on every side (the second-neighbour
 * gradient reaches x +- 2, y +- 2) */
#define GW 2
static size_t gidx(const or_sim *s, int x, int y)
{
    return (size_t)(y + GW) * (size_t)(s->p.nx + 2 * GW) + (size_t)(x + GW);
}

or_sim *or_create(const or_params *p)
{
    if (p->nx < 1 || p->ny < 1) return NULL;
    or_sim *s = (or_sim *)calloc(1, sizeof(or_sim));
    s->p = *p;
    or_alphas(p->rho0_r, p->rho0_b, p->alpha_light, &s->alpha[0], &s->alpha[1]);
    s->rho0[0] = p->rho0_r;
    s->rho0[1] = p->rho0_b;
    for (int k = 0; k < 2; ++k) s->cs2[k] = 3.0 * (1.0 - s->alpha[k]) / 5.0; /* eq. (pressureRelation) */
    s->omega[0] = 1.0 / p->tau_r;
    s->omega[1] = 1.0 / p->tau_b;
    size_t n = (size_t)p->nx * p->ny;
    s->post = (double *)calloc(18 * n, sizeof(double));
    s->strm = (double *)calloc(18 * n, sizeof(double));
    s->rho = (double *)calloc(2 * n, sizeof(double));
    s->ux = (double *)calloc(n, sizeof(double));
    s->uy = (double *)calloc(n, sizeof(double));
    s->psi = (double *)calloc((size_t)(p->nx + 2 * GW) * (p->ny + 2 * GW), sizeof(double));
    s->q = (double *)calloc(4 * (size_t)(p->nx + 2 * GW) * (p->ny + 2 * GW), sizeof(double));
    s->inlet_color = (signed char *)malloc((size_t)p->ny);
    memset(s->inlet_color, 1, (size_t)p->ny);
    return s;
}

void or_destroy(or_sim *s)
{
    if (!s) return;
    free(s->post);
    free(s->strm);
    free(s->rho);
    free(s->ux);
    free(s->uy);
    free(s->psi);
    free(s->q);
    free(s->inlet_color);
    free(s);
}

/* the equilibrium in use: Sec. 2.1.3's Hermite form with the Navier-Stokes
 * correction, else Sec. 2.1.1's */
static void equilibrium(const or_sim *s, double rho_k, double ux, double uy, int k, double *out9)
{
    if (s->p.ns_correction) or_equilibrium_hermite(rho_k, ux, uy, s->alpha[k], out9);
    else or_equilibrium(rho_k, ux, uy, s->alpha[k], out9);
}

/* initial state: equilibrium of the given fields (Sec. 2.1.1 eq. (equilibrium)) */
int or_init(or_sim *s, const double *rho_r, const double *rho_b, const double *ux, const double *uy)
{
    int nx = s->p.nx, ny = s->p.ny;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t c = (size_t)y * nx + x;
            double u = ux ? ux[c] : 0.0, v = uy ? uy[c] : 0.0;
            double e[9];
            equilibrium(s, rho_r[c], u, v, 0, e);
            for (int i = 0; i < 9; ++i) POP(s->post, 0, i, y, x) = e[i];
            equilibrium(s, rho_b[c], u, v, 1, e);
            for (int i = 0; i < 9; ++i) POP(s->post, 1, i, y, x) = e[i];
        }
    s->step = 0;
    return 0;
}

void or_set_inlet_color(or_sim *s, const signed char *color_y)
{
    memcpy(s->inlet_color, color_y, (size_t)s->p.ny);
}

/* Pass 1: streaming, eq. (subop4) as a pull, with periodic wrap and halfway
 * bounce-back at walls (Sec. 2.5 items 1-2). Directions that would come from
 * outside an open x face are filled with the node's own opposite population
 * as a placeholder; pass 2 overwrites them. */
static void pass_stream(or_sim *s)
{
    int nx = s->p.nx, ny = s->p.ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x)
            for (int k = 0; k < 2; ++k)
                for (int i = 0; i < 9; ++i) {
                    int sx = x - CX[i], sy = y - CY[i];
                    int outside = 0, beyond_wall = 0;
                    if (sy < 0 || sy >= ny) {
                        if (s->p.bc_y == OR_BCY_PERIODIC) sy = wrap(sy, ny);
                        else beyond_wall = sy < 0 ? 1 : 2;
                    }
                    if (sx < 0 || sx >= nx) {
                        if (s->p.bc_x == OR_BCX_PERIODIC) sx = wrap(sx, nx);
                        else outside = 1;
                    }
                    int slip = (beyond_wall == 1 && s->p.slip_lo) || (beyond_wall == 2 && s->p.slip_hi);
                    double v;
                    if (beyond_wall && slip && CX[i] != 0 && !outside)
                        /* free slip: the population that left the upstream node of the
                           same row towards the wall, reflected in y only */
                        v = POP(s->post, k, mirror_y(i), y, sx);
                    else if (beyond_wall || outside)
                        /* no slip (link bounce-back); at an open face a placeholder that
                           the Zou-He completion overwrites */
                        v = POP(s->post, k, opposite(i), y, x);
                    else
                        v = POP(s->post, k, i, sy, sx);
                    POP(s->strm, k, i, y, x) = v;
                }
}

/* Pass 2: colour densities, and the two-phase Zou-He completion of the open
 * columns (Sec. 2.5 item 3, R7). */
static void pass_densities_and_open_bc(or_sim *s)
{
    int nx = s->p.nx, ny = s->p.ny;
    size_t n = (size_t)nx * ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x)
            for (int k = 0; k < 2; ++k) {
                double r = 0.0;
                for (int i = 0; i < 9; ++i) r += POP(s->strm, k, i, y, x);
                s->rho[k * n + (size_t)y * nx + x] = r;
            }
    if (s->p.bc_x != OR_BCX_OPEN) return;
    for (int y = 0; y < ny; ++y) {
        /* inlet column x = 0: prescribed colour and velocity */
        {
            int x = 0;
            double N[9];
            for (int i = 0; i < 9; ++i) N[i] = POP(s->strm, 0, i, y, x) + POP(s->strm, 1, i, y, x);
            int red = s->inlet_color[y] > 0;
            double chi[2] = {red ? 1.0 : 0.0, red ? 0.0 : 1.0};
            double vx = red ? s->p.u_in_r : s->p.u_in_b;
            double kap = s->p.ns_correction ? chi[0] * (3.0 * s->cs2[0] - 1.0) + chi[1] * (3.0 * s->cs2[1] - 1.0)
                                            : 0.0;
            double rho_in = or_zouhe_west(N, vx, 0.0, kap);
            static const int unk[3] = {1, 5, 8};
            for (int k = 0; k < 2; ++k) {
                for (int j = 0; j < 3; ++j) POP(s->strm, k, unk[j], y, x) = chi[k] * N[unk[j]];
                s->rho[k * n + (size_t)y * nx + x] = chi[k] * rho_in;
            }
        }
        /* outlet column x = nx-1: prescribed pressure */
        {
            int x = nx - 1;
            static const int known[6] = {0, 1, 2, 4, 5, 8};
            double kn[2] = {0.0, 0.0}, N[9];
            for (int k = 0; k < 2; ++k)
                for (int j = 0; j < 6; ++j) kn[k] += POP(s->strm, k, known[j], y, x);
            double vol_r = kn[0] / s->rho0[0], vol_b = kn[1] / s->rho0[1];
            if (s->p.alt & OR_ALT_OUTLET_UPSTREAM) {
                /* the colour of the node upstream, at this step */
                vol_r = s->rho[(size_t)y * nx + (nx - 2)] / s->rho0[0];
                vol_b = s->rho[n + (size_t)y * nx + (nx - 2)] / s->rho0[1];
            }
            double chi[2] = {vol_r / (vol_r + vol_b), vol_b / (vol_r + vol_b)};
            /* a colour fraction, (phi + 1) / 2 with phi in [-1, 1]: a trace
             * colour whose incoming populations sum below zero has none */
            for (int k = 0; k < 2; ++k) chi[k] = chi[k] < 0.0 ? 0.0 : (chi[k] > 1.0 ? 1.0 : chi[k]);
            double rk[2] = {chi[0] * s->p.p_out / s->cs2[0], chi[1] * s->p.p_out / s->cs2[1]};
            for (int i = 0; i < 9; ++i) N[i] = POP(s->strm, 0, i, y, x) + POP(s->strm, 1, i, y, x);
            double kap = s->p.ns_correction ? chi[0] * (3.0 * s->cs2[0] - 1.0) + chi[1] * (3.0 * s->cs2[1] - 1.0)
                                            : 0.0;
            or_zouhe_east(N, rk[0] + rk[1], 0.0, kap);
            static const int unk[3] = {3, 6, 7};
            for (int k = 0; k < 2; ++k) {
                for (int j = 0; j < 3; ++j) POP(s->strm, k, unk[j], y, x) = chi[k] * N[unk[j]];
                s->rho[k * n + (size_t)y * nx + x] = rk[k];
            }
        }
    }
}

/* Pass 3: velocity, Sec. 2.1.1 momentum sum, with the half-force shift (R4) */
static void pass_velocity(or_sim *s)
{
    int nx = s->p.nx, ny = s->p.ny;
    size_t n = (size_t)nx * ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t c = (size_t)y * nx + x;
            double rho = s->rho[c] + s->rho[n + c], jx = 0.0, jy = 0.0;
            for (int k = 0; k < 2; ++k)
                for (int i = 0; i < 9; ++i) {
                    jx += CX[i] * POP(s->strm, k, i, y, x);
                    jy += CY[i] * POP(s->strm, k, i, y, x);
                }
            s->ux[c] = (jx + 0.5 * rho * s->p.gx) / rho;
            s->uy[c] = (jy + 0.5 * rho * s->p.gy) / rho;
        }
}

/* Sec. 2.1.1 eq. (color_field) */
static double color_field(const or_sim *s, double rho_r, double rho_b)
{
    double a = rho_r / s->rho0[0], b = rho_b / s->rho0[1];
    return (a - b) / (a + b);
}

/* value of a field f (ghost layout, gidx) at (x, y) in [-1, nx] x [-1, ny],
 * ghost rules of R6 */
static double ghost_value(const or_sim *s, const double *f, int x, int y)
{
    int nx = s->p.nx, ny = s->p.ny;
    if (s->p.bc_x == OR_BCX_PERIODIC) x = wrap(x, nx);
    if (s->p.bc_y == OR_BCY_PERIODIC) y = wrap(y, ny);
    int xin = x >= 0 && x < nx, yin = y >= 0 && y < ny;
    if (xin && yin) return f[gidx(s, x, y)];
    if (!yin) {
        /* wall (solid) node: W-weighted mean over fluid neighbours, Sec. 2.4 */
        double num = 0.0, den = 0.0;
        for (int i = 1; i < 9; ++i) {
            int fx = x + CX[i], fy = y + CY[i];
            if (s->p.bc_x == OR_BCX_PERIODIC) fx = wrap(fx, nx);
            if (fx < 0 || fx >= nx || fy < 0 || fy >= ny) continue;
            num += Wt(i) * f[gidx(s, fx, fy)];
            den += Wt(i);
        }
        return num / den;
    }
    /* open-boundary ghost column: nearest in-domain column */
    return f[gidx(s, x < 0 ? 0 : nx - 1, y)];
}

/* fill the ghost cells of f: ghost columns first (they only read the
 * domain), then the ghost rows next to the domain, then the outer ghost
 * rows: periodic wrap, or beyond a wall a copy of the inner ghost row (R15:
 * solid nodes with no fluid neighbour are not defined by Sec. 2.4) */
static void fill_ghosts(const or_sim *s, double *f)
{
    int nx = s->p.nx, ny = s->p.ny;
    for (int y = 0; y < ny; ++y)
        for (int g = 1; g <= GW; ++g) {
            f[gidx(s, -g, y)] = ghost_value(s, f, -g, y);
            f[gidx(s, nx - 1 + g, y)] = ghost_value(s, f, nx - 1 + g, y);
        }
    for (int x = -GW; x < nx + GW; ++x) {
        /* periodic x: the ghost row wraps; beyond an open face the outer
           ghost columns repeat the inner one */
        int xe = s->p.bc_x == OR_BCX_PERIODIC ? x : (x < -1 ? -1 : (x > nx ? nx : x));
        f[gidx(s, x, -1)] = ghost_value(s, f, xe, -1);
        f[gidx(s, x, ny)] = ghost_value(s, f, xe, ny);
    }
    for (int x = -GW; x < nx + GW; ++x) {
        if (s->p.bc_y == OR_BCY_PERIODIC) {
            f[gidx(s, x, -2)] = f[gidx(s, x, wrap(-2, ny))];
            f[gidx(s, x, ny + 1)] = f[gidx(s, x, wrap(ny + 1, ny))];
        } else if (s->p.alt & OR_ALT_ISO_EXTRAP) {
            f[gidx(s, x, -2)] = 2.0 * f[gidx(s, x, -1)] - f[gidx(s, x, 0)];
            f[gidx(s, x, ny + 1)] = 2.0 * f[gidx(s, x, ny)] - f[gidx(s, x, ny - 1)];
        } else {
            f[gidx(s, x, -2)] = f[gidx(s, x, -1)];
            f[gidx(s, x, ny + 1)] = f[gidx(s, x, ny)];
        }
    }
}

/* Pass 4: colour field on the domain, then the ghost layer; with the
 * Navier-Stokes correction also Q^k = (1.8 alpha_k - 0.8) rho_k u of
 * Sec. 2.1.3, its ghost values by the same rules (R14) */
static void pass_color_field(or_sim *s)
{
    int nx = s->p.nx, ny = s->p.ny;
    size_t n = (size_t)nx * ny, g = (size_t)(nx + 2 * GW) * (ny + 2 * GW);
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t c = (size_t)y * nx + x;
            s->psi[gidx(s, x, y)] = color_field(s, s->rho[c], s->rho[n + c]);
        }
    fill_ghosts(s, s->psi);
    if (!s->p.ns_correction) return;
    for (int k = 0; k < 2; ++k) {
        double a = 1.8 * s->alpha[k] - 0.8;
        double *qx = s->q + (2 * k) * g, *qy = s->q + (2 * k + 1) * g;
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t c = (size_t)y * nx + x;
                qx[gidx(s, x, y)] = a * s->rho[k * n + c] * s->ux[c];
                qy[gidx(s, x, y)] = a * s->rho[k * n + c] * s->uy[c];
            }
        fill_ghosts(s, qx);
        fill_ghosts(s, qy);
        if ((s->p.alt & OR_ALT_Q_WALL_ZERO) && s->p.bc_y == OR_BCY_WALLS)
            for (int x = -GW; x < nx + GW; ++x)
                for (int gy = 1; gy <= GW; ++gy) {
                    qx[gidx(s, x, -gy)] = qy[gidx(s, x, -gy)] = 0.0;
                    qx[gidx(s, x, ny - 1 + gy)] = qy[gidx(s, x, ny - 1 + gy)] = 0.0;
                }
    }
}

/* dQx/dx and dQy/dy of colour k at (x, y) with the stencil of
 * eq. (colorGradient) (Sec. 2.1.3) */
static void q_divergence(const or_sim *s, int k, int x, int y, double *dqx, double *dqy)
{
    size_t g = (size_t)(s->p.nx + 2 * GW) * (s->p.ny + 2 * GW);
    double px[9], py[9], Gx[2], Gy[2];
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            size_t o = gidx(s, x + dx, y + dy);
            px[(dy + 1) * 3 + (dx + 1)] = s->q[(2 * k) * g + o];
            py[(dy + 1) * 3 + (dx + 1)] = s->q[(2 * k + 1) * g + o];
        }
    or_gradient3x3(px, Gx);
    or_gradient3x3(py, Gy);
    *dqx = Gx[0];
    *dqy = Gy[1];
}

/* colour gradient at (x, y) from the extended psi field: eq. (colorGradient),
 * or the second-neighbour isotropic stencil (R15); before any wetting turn */
static void node_gradient(const or_sim *s, int x, int y, double *F)
{
    double patch[25];
    for (int dy = -2; dy <= 2; ++dy)
        for (int dx = -2; dx <= 2; ++dx) patch[(dy + 2) * 5 + (dx + 2)] = s->psi[gidx(s, x + dx, y + dy)];
    if (s->p.gradient == 1) {
        or_gradient5x5(patch, F);
    } else {
        double p9[9];
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) p9[(dy + 1) * 3 + (dx + 1)] = patch[(dy + 2) * 5 + (dx + 2)];
        or_gradient3x3(p9, F);
    }
}

/* Pass 5: per node collision (Sec. 2.1), perturbation (Sec. 2.2),
 * recolouring (Sec. 2.3); result into the post-recolouring state. */
static void pass_collide(or_sim *s)
{
    int nx = s->p.nx, ny = s->p.ny;
    size_t n = (size_t)nx * ny;
    const or_params *p = &s->p;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t c = (size_t)y * nx + x;
            double rk[2] = {s->rho[c], s->rho[n + c]};
            double u = s->ux[c], v = s->uy[c];
            double F[2];
            node_gradient(s, x, y, F);
            if (p->bc_y == OR_BCY_WALLS && p->contact_angle >= 0.0 && (y == 0 || y == ny - 1)) {
                /* wetting (Sec. 2.4, R11): the wall normal points into the fluid and
                   the gradient points into red, so the angle between them is the
                   contact angle measured through blue, pi minus red's */
                double ns[2] = {0.0, y == 0 ? 1.0 : -1.0}, Fw[2];
                or_wetting(F, ns, PI_ * (1.0 - p->contact_angle / 180.0), Fw);
                F[0] = Fw[0];
                F[1] = Fw[1];
            }
            double psi = s->psi[gidx(s, x, y)];
            double w = or_omega_eff(psi, s->omega[0], s->omega[1], p->delta);
            double A = p->sigma > 0.0 ? 9.0 * p->sigma * w / 4.0 : p->A;

            /* per colour: populations, equilibria, forcing terms */
            double Nk[2][9], Ek[2][9], Gk[2][9];
            for (int k = 0; k < 2; ++k) {
                for (int i = 0; i < 9; ++i) Nk[k][i] = POP(s->strm, k, i, y, x);
                equilibrium(s, rk[k], u, v, k, Ek[k]);
                for (int i = 0; i < 9; ++i) {
                    /* Guo force density rho_k g (R4) */
                    double cu = CX[i] * u + CY[i] * v;
                    double gxk = rk[k] * p->gx, gyk = rk[k] * p->gy;
                    Gk[k][i] = Wt(i) * ((3.0 * (CX[i] - u) + 9.0 * cu * CX[i]) * gxk +
                                        (3.0 * (CY[i] - v) + 9.0 * cu * CY[i]) * gyk);
                }
            }
            double Nss[9];
            double pert[9];
            or_perturbation(F, A, pert);
            /* Navier-Stokes correction source per colour (Sec. 2.1.3, MRT only) */
            double Uk[2][9] = {{0.0}};
            if (p->ns_correction && p->collision == OR_MRT) {
                double s9[9];
                mrt_rates(w, p->mrt_lambda, s9);
                for (int k = 0; k < 2; ++k) {
                    double dqx, dqy;
                    q_divergence(s, k, x, y, &dqx, &dqy);
                    or_ns_source(dqx, dqy, s9[1], s9[7], Uk[k]);
                }
            }
            if (!p->percolor) {
                /* colour-blind form (R8) */
                double N[9], E[9], G[9], Ns[9];
                for (int i = 0; i < 9; ++i) {
                    N[i] = Nk[0][i] + Nk[1][i];
                    E[i] = Ek[0][i] + Ek[1][i];
                    G[i] = Gk[0][i] + Gk[1][i];
                }
                if (p->collision == OR_BGK) {
                    for (int i = 0; i < 9; ++i) Ns[i] = N[i] - w * (N[i] - E[i]) + (1.0 - w / 2.0) * G[i];
                } else {
                    double s9[9], half[9], Gf[9];
                    or_mrt_collide(N, E, w, p->mrt_lambda, Ns);
                    mrt_rates(w, p->mrt_lambda, s9);
                    for (int j = 0; j < 9; ++j) half[j] = 1.0 - s9[j] / 2.0;
                    mrt_apply(G, half, Gf);
                    for (int i = 0; i < 9; ++i) Ns[i] += Gf[i] + Uk[0][i] + Uk[1][i];
                }
                for (int i = 0; i < 9; ++i) Nss[i] = Ns[i] + pert[i];
            } else {
                /* per-colour form: each colour relaxes to its own equilibrium
                 * and receives A/2 of the perturbation (Sec. 2.2 sum over l != k) */
                for (int i = 0; i < 9; ++i) Nss[i] = 0.0;
                for (int k = 0; k < 2; ++k) {
                    double Ns[9];
                    if (p->collision == OR_BGK) {
                        for (int i = 0; i < 9; ++i)
                            Ns[i] = Nk[k][i] - w * (Nk[k][i] - Ek[k][i]) + (1.0 - w / 2.0) * Gk[k][i];
                    } else {
                        double s9[9], half[9], Gf[9];
                        or_mrt_collide(Nk[k], Ek[k], w, p->mrt_lambda, Ns);
                        mrt_rates(w, p->mrt_lambda, s9);
                        for (int j = 0; j < 9; ++j) half[j] = 1.0 - s9[j] / 2.0;
                        mrt_apply(Gk[k], half, Gf);
                        for (int i = 0; i < 9; ++i) Ns[i] += Gf[i] + Uk[k][i];
                    }
                    for (int i = 0; i < 9; ++i) Nss[i] += Ns[i] + 0.5 * pert[i];
                }
            }
            double outr[9], outb[9];
            or_recolor(Nss, rk[0], rk[1], F, p->beta, s->alpha[0], s->alpha[1], outr, outb);
            for (int i = 0; i < 9; ++i) {
                POP(s->post, 0, i, y, x) = outr[i];
                POP(s->post, 1, i, y, x) = outb[i];
            }
        }
}

static void macro_passes(or_sim *s)
{
    pass_stream(s);
    pass_densities_and_open_bc(s);
    pass_velocity(s);
}

void or_step(or_sim *s, long nsteps)
{
    for (long t = 0; t < nsteps; ++t) {
        macro_passes(s);
        pass_color_field(s);
        pass_collide(s);
        s->step++;
    }
}

/* moments of the streamed, boundary-completed state; p from eq. (pressureRelation) */
void or_moments(or_sim *s, double *rho_r, double *rho_b, double *ux, double *uy, double *p)
{
    int nx = s->p.nx, ny = s->p.ny;
    size_t n = (size_t)nx * ny;
    macro_passes(s);
    for (size_t c = 0; c < n; ++c) {
        if (rho_r) rho_r[c] = s->rho[c];
        if (rho_b) rho_b[c] = s->rho[n + c];
        if (ux) ux[c] = s->ux[c];
        if (uy) uy[c] = s->uy[c];
        if (p) p[c] = s->rho[c] * s->cs2[0] + s->rho[n + c] * s->cs2[1];
    }
}

void or_gradients(or_sim *s, double *Fx, double *Fy, double *dqxdx, double *dqydy)
{
    int nx = s->p.nx, ny = s->p.ny;
    size_t n = (size_t)nx * ny;
    macro_passes(s);
    pass_color_field(s);
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t c = (size_t)y * nx + x;
            double F[2];
            node_gradient(s, x, y, F);
            if (Fx) Fx[c] = F[0];
            if (Fy) Fy[c] = F[1];
            for (int k = 0; k < 2 && s->p.ns_correction; ++k) {
                double dqx, dqy;
                q_divergence(s, k, x, y, &dqx, &dqy);
                if (dqxdx) dqxdx[k * n + c] = dqx;
                if (dqydy) dqydy[k * n + c] = dqy;
            }
        }
}

void or_get_pops(const or_sim *s, double *out)
{
    memcpy(out, s->post, 18 * (size_t)s->p.nx * s->p.ny * sizeof(double));
}

void or_set_pops(or_sim *s, const double *in)
{
    memcpy(s->post, in, 18 * (size_t)s->p.nx * s->p.ny * sizeof(double));
}

/* A storage model, not part of the method: each stored population rounded
 * to the nearest FP32 number, which is what FP32 storage alone does to the
 * FP64 state after a step.  The parity tests measure with it how much the
 * flow amplifies rounding. */
void or_round_f32(or_sim *s)
{
    long n = 18 * (long)s->p.nx * s->p.ny;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < n; ++c)
        s->post[c] = (double)(float)s->post[c];
}

long or_step_count(const or_sim *s) { return s->step; }

int or_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
