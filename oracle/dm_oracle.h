/*
 * dm_oracle.h -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 * Declarations of the plain FP64 CPU oracle in dm_oracle.c.  Only tests/,
 * __graft_entry__.smoke() and bench.py's cpu_baseline leg use it.
 */
#ifndef DM_ORACLE_H
#define DM_ORACLE_H
#include <stdint.h>

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4]);
void orc_gauss4(uint64_t seed, uint32_t block, uint32_t chain, int64_t step,
                uint32_t comp, uint32_t tag, double z[4]);
double orc_normal(uint64_t seed, uint32_t index, uint32_t chain, int64_t step,
                  uint32_t comp, uint32_t tag);
void orc_reduced_params(double lambda, double kappa, double kT, double a,
                        double xi, double *T_star, double *nu, double *b,
                        double *d, double *time_unit);
void orc_tables(int M, double nu, double T_star, double dtau, double *phi,
                double *zeta_l, double *zeta, double *E, double *C, double *W);
void orc_modes_from_positions(int M, const double *phi, const double *pos,
                              double *R);
void orc_positions_from_modes(int M, const double *phi, const double *R,
                              double *pos);
void orc_delta_h(int M, double nu, const double *R, double *dH);
void orc_step_modes(int M, int n_chains, const uint32_t *chain_id, double *R,
                    double nu, double T_star, double dtau, double gamma_dot,
                    int nonlinear, uint64_t seed, int64_t step0,
                    int64_t n_steps);
void orc_bead_force(int M, double nu, const double *pos, double *f);
void orc_step_euler(int M, int n_chains, const uint32_t *chain_id, double *pos,
                    double nu, double T_star, double dtau, double gamma_dot,
                    uint64_t seed, int64_t step0, int64_t n_steps);
double orc_energy(int M, double nu, const double *pos);
void orc_set_threads(int n);
void orc_step_wlc(int M, int n_chains, const uint32_t *chain_id, double *pos,
                  double T_bar, double dt, int iters, double tol, int midpoint,
                  uint64_t seed, int64_t step0, int64_t n_steps);
void orc_mc_sweeps(int M, int n_chains, const uint32_t *chain_id, double *R,
                   double nu, double T_star, double scale, uint64_t seed,
                   int64_t step0, int64_t n_sweeps, int64_t *accepted);
void orc_chain_observables(int M, const double *pos, double *out);
void orc_config_chains(int M, int n_chains, const uint32_t *chain_id, double b,
                       uint64_t seed, double *pos);

#endif
