/*
 * dg_oracle.h -- interface of the plain FP64 CPU oracle (test infrastructure
 * only; see dg_oracle.c).  Host arrays only.  State layout:
 * w[cell][field][mode], cell = i + n0 (j + n1 k), mode = l_x + p (l_y + p l_z),
 * fields (rho, rho v_x, rho v_y[, rho v_z], e[, c rho][, alpha]).
 */
#ifndef DG_ORACLE_H
#define DG_ORACLE_H

typedef struct {
    int dim;           /* 2 or 3 */
    int n[3];          /* cells per axis */
    int bc[3];         /* 0 periodic, 1 outflow (mirrored ghost), 2 reflecting wall */
    double h;          /* cubic cell size */
    int order;         /* p = n + 1 modes and Gauss points per axis */
    double gamma, nu, kappa;
    int av_on;
    double av_scale, f_v, f_tau, f_w, s_onset, alpha_max;
    double cfl;
    const double *forcing; /* [cell][3][p^d] coefficients of s, or NULL */
    int limiter;       /* positivity limiter after every RK stage (Sec. 4.2) */
    int tracer;        /* passive tracer field c rho after e (Sec. 3.4) */
    double eta;        /* its diffusivity */
    int basis;         /* 0 tensor set Q_n, 1 total-degree set P_n (Sec. 2.3) */
} or_params;

void or_legendre(int lmax, double x, double *Pt, double *dPt);
void or_gauss(int n, double *x, double *w);
void or_euler_flux(int d, double gamma, const double *u, int a, double *f);
void or_hllc(int d, double gamma, const double *uL, const double *uR, int a, double *F);
double or_recovery_fraction(int order);
void or_recover_face(const or_params *pr, const double *wL, const double *wR, int a, double *ut, double *gt);
double or_sensor(int p, int d, const double *wrho);
double or_sensor_rate(int p, int d, const double *wrho, const double *wdrho);
void or_rhs(const or_params *pr, const double *w, const double *R_prev, double *wdot, double *R_out);
void or_rhs_cells(const or_params *pr, const double *w, const double *R_prev, long ncells_sel, const long *cells,
                  double *out);
void or_rhs_abs(const or_params *pr, const double *w, const double *R_prev, long ncells_sel, const long *cells,
                double *out);
double or_max_dt(const or_params *pr, const double *w, double *cmax_out, double *vmax_out);
int or_rk_stages(int order);
void or_step(const or_params *pr, double *w, double dt, double *R_state);
void or_totals(const or_params *pr, const double *w, double *out);
long or_limit(const or_params *pr, double *w);
int or_n_modes(int p, int d, int basis);
void or_mode_degrees(int p, int d, int basis, int m, int *l);
int or_forcing_modes(int dim, int kmax, int *kv);
void or_ou_update(int dim, int nm, const int *kv, double *amp, const double *noise, double dt, double t_corr,
                  double sigma0);
void or_forcing_project(const or_params *pr, const double *lo, int nm, const int *kv, const double *amp,
                        double *s);
int or_num_threads(void);
void or_set_num_threads(int n);

#endif
