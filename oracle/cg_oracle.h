/*
 * cg_oracle.h -- plain FP64 CPU oracle of the two-population colour-gradient
 * lattice Boltzmann step (D2Q9), Douillet-Grellier et al., arXiv:1903.01168,
 * Section 2 ("LBM immiscible multiphase model") and Appendix B.
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no source,
 * header, table or helper with the HIP implementation.  It is slow on purpose:
 * every sub-step of the paper is a separate full-lattice pass in FP64.
 *
 * Conventions (identical to the public C ABI, restated here independently):
 *  - host arrays are row-major [ny][nx], x fastest, y pointing "north";
 *  - populations are stored per colour: pop[k][i][y][x], k=0 red, k=1 blue;
 *  - the stored state is the post-recolouring population of the last step
 *    (about to be streamed); the initial state is the equilibrium of the
 *    given fields;
 *  - the macroscopic fields "at step n" are the moments of the streamed and
 *    boundary-completed populations, i.e. what step n+1 collides.
 */
#ifndef CG_ORACLE_H
#define CG_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_BCX_PERIODIC = 0, OR_BCX_OPEN = 1 };   /* open: velocity inlet at x=0, pressure outlet at x=nx-1 */
enum { OR_BCY_PERIODIC = 0, OR_BCY_WALLS = 1 };  /* walls: halfway (link) reflection, see slip_lo/hi */
enum { OR_BGK = 0, OR_MRT = 1 };

typedef struct {
    int nx, ny;
    int bc_x, bc_y;
    int collision;          /* OR_BGK or OR_MRT */
    int percolor;           /* 1: collide and perturb each colour separately (check of the colour-blind form) */
    double rho0_r, rho0_b;  /* reference densities */
    double alpha_light;     /* alpha of the lighter fluid (0.2 in the paper) */
    double tau_r, tau_b;    /* relaxation times, tau = 3 nu + 1/2 */
    double delta;           /* interface width of the omega interpolation (0.1) */
    double A;               /* constant perturbation amplitude, or 0 */
    double sigma;           /* surface tension: A(x) = 9 sigma omega_eff(x) / 4, or 0 */
    double beta;            /* recolouring parameter */
    double mrt_lambda;      /* s_0..s_6 = lambda * omega_eff (4/5) */
    double gx, gy;          /* body force per unit mass */
    double u_in_r, u_in_b;  /* inlet x-velocity of a red / blue inlet node */
    double p_out;           /* outlet pressure */
    int slip_lo, slip_hi;   /* walls: 0 no-slip (bounce-back), 1 free-slip (specular reflection,
                               Sec. 2.5 item 1) at y = -1/2 and y = ny - 1/2 */
    double contact_angle;   /* walls: static contact angle of the red fluid, measured through red,
                               in degrees (Sec. 2.4); < 0: no adjustment of the colour gradient */
    int ns_correction;      /* 1: Sec. 2.1.3 Navier-Stokes correction (Hermite equilibrium everywhere,
                               the MRT source U^k, Hermite terms of the Zou-He completion) */
    int gradient;           /* 0: eq. (colorGradient), nearest neighbours; 1: the second-neighbour
                               8th-order isotropic stencil (R15) */
    int alt;                /* alternative readings of rules the paper leaves open, for measuring how
                               much they matter (0: the readings R1-R15 used everywhere); bits: */
} or_params;

/* or_params.alt bits */
enum {
    OR_ALT_Q_WALL_ZERO = 1,     /* R14: Q ghost values beyond a wall are 0 (the wall is at rest) instead of
                                   the colour field's extrapolation */
    OR_ALT_ISO_EXTRAP = 2,      /* R15: the outer ghost row beyond a wall is the linear extrapolation
                                   2 g - f of the inner ghost row g and the wall row f, not a copy of g */
    OR_ALT_OUTLET_UPSTREAM = 4  /* R7: outlet colour fractions from the colour field of the node upstream
                                   (x = nx - 2) at this step, not from the six populations streaming in */
};

typedef struct or_sim or_sim;

/* ---- node-level operators (exported so that tests can pin them) ---- */
void   or_lattice(int *cx, int *cy, int *opp, double *W);        /* 9 each */
void   or_tables(double alpha, double *phi, double *B, double *xi); /* 9 each */
void   or_alphas(double rho0_r, double rho0_b, double alpha_light, double *alpha_r, double *alpha_b);
void   or_equilibrium(double rho_k, double ux, double uy, double alpha_k, double *out9);
double or_omega_eff(double psi, double omega_r, double omega_b, double delta);
void   or_gradient3x3(const double *psi9, double *F2);   /* psi9[(dy+1)*3+(dx+1)] */
void   or_gradient5x5(const double *psi25, double *F2);  /* psi25[(dy+2)*5+(dx+2)] */
void   or_equilibrium_hermite(double rho_k, double ux, double uy, double alpha_k, double *out9);
/* Sec. 2.1.3: U = M^{-1} C from dQx/dx, dQy/dy and the rates s_1, s_7 */
void   or_ns_source(double dQxdx, double dQydy, double s1, double s7, double *out9);
void   or_perturbation(const double *F2, double A, double *out9); /* the added term */
/* Sec. 2.4: the colour gradient F2 of a fluid node next to a wall with unit
 * normal ns (pointing into the fluid) turned to make the angle theta (radians,
 * measured between the gradient and ns) with the wall: the closer of the two
 * candidates, its length kept. */
void   or_wetting(const double *F2, const double *ns2, double theta, double *out2);
void   or_recolor(const double *Nss9, double rho_r, double rho_b, const double *F2, double beta,
                  double alpha_r, double alpha_b, double *out_r9, double *out_b9);
double or_zouhe_west(double *N9, double vx, double vy, double kap);   /* completes 1,5,8; returns rho */
double or_zouhe_east(double *N9, double rho, double vy, double kap);  /* completes 3,6,7; returns v_x */
/* kap: 0 with the equilibrium of Sec. 2.1.1; sum_k chi_k (3 c_s,k^2 - 1) with
 * the Hermite equilibrium of Sec. 2.1.3 (Sec. 2.5 item 3, term H) */
void   or_mrt_matrices(double *M81, double *Minv81);
void   or_mrt_collide(const double *N9, const double *Neq9, double omega, double lambda, double *out9);

/* ---- lattice-level driver ---- */
or_sim *or_create(const or_params *p);
void    or_destroy(or_sim *s);
int     or_init(or_sim *s, const double *rho_r, const double *rho_b, const double *ux, const double *uy);
void    or_set_inlet_color(or_sim *s, const signed char *color_y); /* +1 red, -1 blue, per row */
void    or_step(or_sim *s, long nsteps);
void    or_moments(or_sim *s, double *rho_r, double *rho_b, double *ux, double *uy, double *p);
void    or_get_pops(const or_sim *s, double *out);      /* [2][9][ny][nx] */
/* The gradients the next step would use, from the stored state (the state is
 * not advanced): the colour gradient F ([ny][nx] each, before any contact-
 * angle turn) and, with the Navier-Stokes correction, dQx/dx and dQy/dy of
 * each colour ([2][ny][nx] each; NULL to skip). */
void    or_gradients(or_sim *s, double *Fx, double *Fy, double *dqxdx, double *dqydy);
void    or_set_pops(or_sim *s, const double *in);
/* Round the stored populations to FP32 (a storage model for measuring how
 * the flow amplifies rounding; no step of the method). */
void    or_round_f32(or_sim *s);
long    or_step_count(const or_sim *s);
int     or_threads(void);

#ifdef __cplusplus
}
#endif
#endif
