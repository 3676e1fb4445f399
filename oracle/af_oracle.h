/*
 * af_oracle.h -- plain FP64 CPU oracle of the compact fourth-order
 * positivity-preserving Active Flux (AF) method for the 1D/2D compressible
 * Navier-Stokes equations (Duan, Barsukow, Klingenberg).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP path.  It
 * may be loaded by the test suite, by the smoke check and by the CPU-baseline
 * leg of the benchmark, and by nothing else.  It shares no code, header,
 * table or helper with the HIP library; the two are written independently
 * from the paper.
 *
 * State layout (identical to the product library's documented layout, since
 * both are fed the same input buffers):
 *   1D: [avg: 3 x n][pts: 3 x np]          np = n (periodic) or n+1
 *       component-major, point k sits at x0 + k*dx, cell i spans
 *       [x0+i*dx, x0+(i+1)*dx].
 *   2D: [avg: 4 x n2 x n1][xe: 4 x n2 x n1x][ye: 4 x n2y x n1][co: 4 x n2y x n1x]
 *       n1x = n1 (x periodic) or n1+1, n2y likewise; x fastest.
 *       xe(i,j) sits at (x0+i dx, y0+(j+1/2) dy)   (x-face midpoints)
 *       ye(i,j) sits at (x0+(i+1/2) dx, y0+j dy)   (y-face midpoints)
 *       co(i,j) sits at (x0+i dx, y0+j dy)         (cell corners)
 *   Components: 1D (rho, rho u, E); 2D (rho, rho u, rho v, E).
 */
#ifndef AF_ORACLE_H
#define AF_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* boundary kinds (per side: x-low, x-high, y-low, y-high) */
enum { ORC_PERIODIC = 0, ORC_OUTFLOW = 1, ORC_NOSLIP = 2, ORC_SYMMETRY = 3,
       ORC_DIRICHLET = 4 /* 1D only: ghost cells and the boundary point hold bcstate */ };

/* limiter switches */
enum {
  ORC_LIM_SMOOTH = 1,  /* smoothness-indicator blend theta^s            */
  ORC_LIM_PP = 2,      /* density/pressure limiting of cell-average fluxes */
  ORC_LIM_POINT = 4,   /* scaling limiter of point values                 */
  ORC_LIM_CENTRE = 8,  /* scaling limiter of reconstructed centre values  */
  ORC_LIM_LOWONLY = 16, /* diagnostic: low-order LLF cell fluxes and, with
                           ORC_LIM_POINT, low-order point values          */
  ORC_LIM_PEXACT = 64   /* theta^p as the root of the pressure quadratic
                           (reading R-pquad) in place of the linear rule  */
};

/* status flags raised by one forward-Euler stage */
enum {
  ORC_FLAG_CELL_LOW = 1,  /* a low-order cell intermediate state is not admissible  */
  ORC_FLAG_POINT_LOW = 2, /* a low-order point state is not admissible              */
  ORC_FLAG_NONFINITE = 4  /* a non-finite value in the stage output                  */
};

typedef struct orc_cfg {
  int dim;              /* 1 or 2 */
  int n1, n2;           /* cells per axis (n2 unused in 1D) */
  double x0, x1, y0, y1;
  double gamma, mu, Pr;
  double Cs;            /* smoothness-limiter strength (paper: 1) */
  double cfl_c, cfl_v;  /* CFL numbers of the inviscid and viscous parts */
  int limiter;          /* ORC_LIM_* bits */
  int bc[4];            /* x-low, x-high, y-low, y-high */
  int max_halvings;
  int rk;               /* time integrator: 3 (SSP-RK3) or 54 (SSP-RK54) */
  double bcstate[2][3]; /* 1D Dirichlet states (rho, rho u, E), x-low and x-high */
} orc_cfg;

/* sizes (in doubles) */
long orc_state_len(const orc_cfg* c);

/* forward-Euler stage with all enabled limiters: Ufe = FE(U, dt).
 * theta_out (optional, may be NULL): per face [dir][4 comps unused]... see .c */
int orc_fe(const orc_cfg* c, const double* U, double dt, double* Ufe,
           double* theta_s_out, double* theta_pp_out);

/* 2D forward-Euler stage whose cell-average fluxes use a given blend
 * coefficient per face in place of the smoothness blend theta^s: the
 * density/pressure limiter (Sec. 3.3) acts on the candidate
 * F^L + theta_nn (F^H - F^L), so F = F^L + theta_nn theta^rho theta^p
 * (F^H - F^L), never above theta_nn and always admissible.  With theta_nn =
 * theta^s this is the plain stage.  theta_nn has orc_nfaces() entries: x-faces [n2][n1+1]
 * then y-faces [n2+1][n1]; on a periodic axis the last face of a line is the
 * first one again and takes its entry.  Returns the flags, or -1 for a 1D
 * config. */
int orc_fe_blend(const orc_cfg* c, const double* U, double dt, const double* theta_nn,
                 double* Ufe, double* theta_s_out, double* theta_pp_out);

/* faces of the grid: 1D n1+1; 2D x-faces n2*(n1+1) plus y-faces (n2+1)*n1 */
long orc_nfaces(const orc_cfg* c);

/* 2D: the 40 features of the learned blend coefficient of every face
 * (feat[face][40], faces ordered as above); see the .c file for their
 * definition.  Returns -1 for a 1D config. */
int orc_blend_features(const orc_cfg* c, const double* U, double* feat);

/* unlimited semi-discrete right-hand side dU/dt (cell averages and points) */
void orc_rhs(const orc_cfg* c, const double* U, double* dUdt);

/* CFL time step over cell averages */
double orc_dt(const orc_cfg* c, const double* U);

/* the positivity theorem's sufficient time step (end of Sec. 3.4): the
 * intermediate-state bound of the low-order LLF scheme (Sec. 3.1) for the cell
 * averages (under ORC_LIM_PP) and for the low-order point scheme on the half
 * lattice (under ORC_LIM_POINT); +infinity if neither switch is set */
double orc_dt_pp(const orc_cfg* c, const double* U);

/* one step with the halving retry, by SSP-RK3 or (c->rk == 54) the
 * five-stage fourth-order SSP method Sec. 2.3 names.  dt<=0 -> CFL dt.  dt is
 * clipped to t_final - t.  Returns 0 on success, nonzero if max_halvings
 * exceeded. */
int orc_step(const orc_cfg* c, double* U, double dt, double t, double t_final,
             double* dt_used, int* halvings, int* flags_out);

/* run from t0 to t_final (or max_steps); returns 0 or the failing status */
int orc_run(const orc_cfg* c, double* U, double t0, double t_final,
            long max_steps, long* nsteps, double* t_out);

/* building blocks exposed for property tests */
double orc_Theta(double zL, double zH, double eps);
/* theta^p of the exact rule from UL toward UT (reading R-pquad) */
double orc_theta_p_root(const orc_cfg* c, const double* UL, const double* UT, double eps);
double orc_pressure(const orc_cfg* c, const double* U);
void orc_flux_c(const orc_cfg* c, int dir, const double* U, double* F);
void orc_flux_v(const orc_cfg* c, int dir, const double* U, const double* S,
                double* F);
double orc_bvisc(const orc_cfg* c, int dir, const double* U, const double* S);
double orc_op_dplus(const double* z, double dx);
double orc_op_dminus(const double* z, double dx);
double orc_op_dc(const double* z, double dx);
double orc_op_d2(const double* k, const double* z, double dx);
int orc_threads(void);
/* threads of the OpenMP loops of later calls (n >= 1) */
void orc_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
