/*
 * dm_oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * A plain, slow, obviously-correct FP64 CPU implementation of the
 * mode-amplitude Langevin time step of Panja, Barkema & van Leeuwen,
 * "Efficient simulation of semiflexible polymers" (arXiv:1411.3487), and of
 * the bead-space Euler scheme the paper uses as its default method.
 *
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
 * load this file's shared library.  It shares no code, header, table or
 * constant with the HIP library in paper_1411_3487_amd/; both sides implement
 * Philox4x32-10 independently from its publication (Salmon, Moraes, Dror &
 * Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11).
 *
 * Units are the paper's reduced ones (Sec. III, Eqs. b3-b5): lengths in d, time
 * in xi/lambda, noise variance 2 T*.
 *
 * Array layout: a chain's positions or mode amplitudes are 3*M doubles,
 * component-major: x[alpha*M + i], alpha = 0,1,2 (x,y,z), i = bead n or mode
 * p.  Several chains are stored back to back.
 *
 * Readings of the paper taken here (the paper is silent or garbled there):
 *  - phi_{n,0} = 1/sqrt(M), not sqrt(2/M) as Eq. (c8) prints; only then is
 *    phi orthogonal, Eq. (c2).  Modes run p = 0..M-1 (M = N+1 beads).
 *  - The sign of H_p is + dL_c/dR_p, as in Eq. (e1).
 *  - The decay rate of the coupling integral (f0) is zeta_p of Eq. (e9).
 *  - p = 0 has zeta = zeta^l = 0 and Delta H_0 = 0: the centre-of-mass mode
 *    is a random walk with variance 2 T* dtau per component and step.
 *  - Shear (Eq. btum) enters each mode as R^x_p += gdot*dtau*E_p*R^y_p(old),
 *    the exact integrating-factor solution of the drift for R^y decaying at
 *    zeta_p over the step; the x-y noise cross term is neglected.
 *  - Noise: Philox4x32-10, key = (seed lo, seed hi), counter =
 *    (index/4, chain, step lo, (step hi << 8) | (component << 4) | tag);
 *    the four outputs give uniforms (x + 1/2) 2^-32 and two Box-Muller
 *    pairs, normal j of the block goes to index 4*(index/4) + j.
 *    Tags: 0 = mode step, 1 = Euler step.
 *
 * Parity unpinned: the coupling-integral approximation (f1)-(f2) has no
 * closed form; it is pinned only through its small-step limit and the
 * equilibrium statistics the tests check.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "dm_oracle.h"

#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads of the OpenMP loops over chains (timing only: results do not
   depend on it, every chain is computed the same way by one thread). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al. 2011): ten rounds of a multiply-xor         */
/* bijection on a 128-bit counter, with a Weyl-sequence key schedule.       */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                       uint32_t out[4])
{
    const uint32_t mul_a = 0xD2511F53u, mul_b = 0xCD9E8D57u;
    const uint32_t weyl_a = 0x9E3779B9u, weyl_b = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += weyl_a;
            k1 += weyl_b;
        }
        uint64_t pa = (uint64_t)mul_a * (uint64_t)c0;
        uint64_t pb = (uint64_t)mul_b * (uint64_t)c2;
        uint32_t pa_hi = (uint32_t)(pa >> 32), pa_lo = (uint32_t)pa;
        uint32_t pb_hi = (uint32_t)(pb >> 32), pb_lo = (uint32_t)pb;
        uint32_t n0 = pb_hi ^ c1 ^ k0;
        uint32_t n1 = pb_lo;
        uint32_t n2 = pa_hi ^ c3 ^ k1;
        uint32_t n3 = pa_lo;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Four standard normals for the noise block (index/4) of one component. */
void orc_gauss4(uint64_t seed, uint32_t block, uint32_t chain, int64_t step,
                uint32_t comp, uint32_t tag, double z[4])
{
    uint64_t k = (uint64_t)step;
    uint32_t ctr[4] = {block, chain, (uint32_t)k,
                       (uint32_t)((k >> 32) << 8) | (comp << 4) | tag};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    const double two_m32 = 1.0 / 4294967296.0;
    const double two_pi = 6.283185307179586476925286766559;
    double u[4];
    for (int j = 0; j < 4; ++j) u[j] = ((double)x[j] + 0.5) * two_m32;
    double ra = sqrt(-2.0 * log(u[0])), rb = sqrt(-2.0 * log(u[2]));
    z[0] = ra * cos(two_pi * u[1]);
    z[1] = ra * sin(two_pi * u[1]);
    z[2] = rb * cos(two_pi * u[3]);
    z[3] = rb * sin(two_pi * u[3]);
}

double orc_normal(uint64_t seed, uint32_t index, uint32_t chain, int64_t step,
                  uint32_t comp, uint32_t tag)
{
    double z[4];
    orc_gauss4(seed, index / 4u, chain, step, comp, tag, z);
    return z[index % 4u];
}

/* ------------------------------------------------------------------------ */
/* Initial state of the batched workloads (the paper prescribes none): each */
/* chain straight, its beads b apart along a direction e uniform on the     */
/* unit sphere, every coordinate jittered by 0.01 b times a standard normal.*/
/* Philox, step 0: tag 5 block (0, chain, 0, comp 0) gives the direction    */
/* from its first two uniforms, cos(theta) = 2 U0 - 1, phi = 2 pi U1;       */
/* tag 4 gives the jitter, normal index = bead n, component a.              */
/* ------------------------------------------------------------------------ */
void orc_config_chains(int M, int n_chains, const uint32_t *chain_id, double b,
                       uint64_t seed, double *pos)
{
    const double two_m32 = 1.0 / 4294967296.0;
    const double two_pi = 6.283185307179586476925286766559;
    for (int c = 0; c < n_chains; ++c) {
        uint32_t ctr[4] = {0u, chain_id[c], 0u, 5u};
        uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
        uint32_t x[4];
        orc_philox4x32_10(ctr, key, x);
        double u0 = ((double)x[0] + 0.5) * two_m32, u1 = ((double)x[1] + 0.5) * two_m32;
        double ct = 2.0 * u0 - 1.0, st = sqrt(1.0 - ct * ct), ph = two_pi * u1;
        double e[3] = {st * cos(ph), st * sin(ph), ct};
        double *r = pos + (size_t)c * 3 * M;
        for (int a = 0; a < 3; ++a)
            for (int n = 0; n < M; ++n)
                r[a * M + n] = n * b * e[a] +
                               0.01 * b * orc_normal(seed, (uint32_t)n, chain_id[c], 0, (uint32_t)a, 4u);
    }
}

/* ------------------------------------------------------------------------ */
/* Model parameters, Sec. II (Eqs. a2, a3) and Sec. VII.B (Eq. g2).             */
/* ------------------------------------------------------------------------ */
void orc_reduced_params(double lambda, double kappa, double kT, double a,
                        double xi, double *T_star, double *nu, double *b,
                        double *d, double *time_unit)
{
    /* nu = kappa/lambda; b = 1/(1-2 nu) and a = b d (Eq. a3);
       T* = kT/(lambda d^2); t = (xi/lambda) tau (Sec. III). */
    double n_ = kappa / lambda;
    double b_ = 1.0 / (1.0 - 2.0 * n_);
    double d_ = a / b_;
    *nu = n_;
    *b = b_;
    *d = d_;
    *T_star = kT / (lambda * d_ * d_);
    *time_unit = xi / lambda;
}

/* ------------------------------------------------------------------------ */
/* Mode tables for one chain length: Eqs. (c8), (c9), (e9), (d3), (d6),     */
/* (f2).  phi is row-major phi[n*M + p].                                    */
/* ------------------------------------------------------------------------ */
void orc_tables(int M, double nu, double T_star, double dtau, double *phi,
                double *zeta_l, double *zeta, double *E, double *C,
                double *W)
{
    const double pi = 3.141592653589793238462643383279502884;
    for (int n = 0; n < M; ++n)
        for (int p = 0; p < M; ++p) {
            double norm = (p == 0) ? sqrt(1.0 / M) : sqrt(2.0 / M);
            phi[n * M + p] = norm * cos(p * (n + 0.5) * pi / M);
        }
    for (int p = 0; p < M; ++p) {
        double cp = cos(p * pi / M);
        double sp = sin(p * pi / (2.0 * M));
        /* Eq. (c9): longitudinal (Rouse) eigenvalue. */
        double zl = 2.0 * (1.0 - cp) * (1.0 - 2.0 * nu * cp);
        /* Eq. (e9): the decay rate left after moving the linear part of the
           coupling, (1-2nu) [2 sin(p pi / 2M)]^2 R_p, to the left side. */
        double z = zl - (1.0 - 2.0 * nu) * (2.0 * sp) * (2.0 * sp);
        if (p == 0) {
            zl = 0.0;
            z = 0.0;
        }
        zeta_l[p] = zl;
        zeta[p] = z;
        /* Eq. (d3): exact decay of the free mode over one step. */
        E[p] = exp(-z * dtau);
        /* Eq. (f2): [exp(-z dtau) - exp(-zl dtau)] / (zl - z), written as
           exp(-z dtau) * [1 - exp(-(zl-z) dtau)] / (zl - z) with expm1;
           its zl -> z limit is dtau exp(-z dtau) (Eq. f3 for small p). */
        double dz = zl - z;
        C[p] = (dz > 0.0) ? -E[p] * expm1(-dz * dtau) / dz : dtau * E[p];
        /* Eq. (d6): variance T* [1 - exp(-2 z dtau)] / z, limit 2 T* dtau. */
        W[p] = (z > 0.0) ? sqrt(-T_star * expm1(-2.0 * z * dtau) / z)
                         : sqrt(2.0 * T_star * dtau);
    }
}

/* Eq. (c1): R_p = sum_n r_n phi_{n,p}. */
void orc_modes_from_positions(int M, const double *phi, const double *pos,
                              double *R)
{
    for (int a = 0; a < 3; ++a)
        for (int p = 0; p < M; ++p) {
            double s = 0.0;
            for (int n = 0; n < M; ++n) s += pos[a * M + n] * phi[n * M + p];
            R[a * M + p] = s;
        }
}

/* Eq. (c1): r_n = sum_p phi_{n,p} R_p, over p >= p_first. */
static void positions_from_modes(int M, const double *phi, const double *R,
                                 int p_first, double *pos)
{
    for (int a = 0; a < 3; ++a)
        for (int n = 0; n < M; ++n) {
            double s = 0.0;
            for (int p = p_first; p < M; ++p)
                s += phi[n * M + p] * R[a * M + p];
            pos[a * M + n] = s;
        }
}

void orc_positions_from_modes(int M, const double *phi, const double *R,
                              double *pos)
{
    positions_from_modes(M, phi, R, 0, pos);
}

/* Nonlinear part of the coupling, Eqs. (e4), (e11), via the bead force:
   u_n = r_n - r_{n-1}; g_n = u_n (1/|u_n| - (1-2nu)) for bonds n = 1..M-1;
   F_n = g_n - g_{n+1} with g_0 = g_M = 0; Delta H_p = sum_n phi_{n,p} F_n.
   r are positions without the p = 0 mode (forces are translation
   invariant).  dH[a*M + p], dH_0 is returned as computed. */
static void delta_h_from_positions(int M, const double *phi, double nu,
                                   const double *r, double *g, double *F,
                                   double *dH)
{
    const double lin = 1.0 - 2.0 * nu;
    for (int n = 1; n < M; ++n) {
        double u[3], l2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            u[a] = r[a * M + n] - r[a * M + n - 1];
            l2 += u[a] * u[a];
        }
        double l = sqrt(l2);
        for (int a = 0; a < 3; ++a) g[a * M + n] = u[a] * (1.0 / l - lin);
    }
    for (int a = 0; a < 3; ++a) {
        g[a * M + 0] = 0.0; /* g_0 = 0; g_M handled below */
        for (int n = 0; n < M; ++n) {
            double gn = (n >= 1) ? g[a * M + n] : 0.0;
            double gn1 = (n + 1 <= M - 1) ? g[a * M + n + 1] : 0.0;
            F[a * M + n] = gn - gn1;
        }
        for (int p = 0; p < M; ++p) {
            double s = 0.0;
            for (int n = 0; n < M; ++n) s += phi[n * M + p] * F[a * M + n];
            dH[a * M + p] = s;
        }
    }
}

void orc_delta_h(int M, double nu, const double *R, double *dH)
{
    double *phi = malloc(sizeof(double) * M * M);
    double *zl = malloc(sizeof(double) * M), *z = malloc(sizeof(double) * M);
    double *E = malloc(sizeof(double) * M), *C = malloc(sizeof(double) * M);
    double *W = malloc(sizeof(double) * M);
    double *r = malloc(sizeof(double) * 3 * M), *g = malloc(sizeof(double) * 3 * M);
    double *F = malloc(sizeof(double) * 3 * M);
    orc_tables(M, nu, 1.0, 1.0, phi, zl, z, E, C, W);
    positions_from_modes(M, phi, R, 1, r);
    delta_h_from_positions(M, phi, nu, r, g, F, dH);
    free(phi); free(zl); free(z); free(E); free(C); free(W);
    free(r); free(g); free(F);
}

/* ------------------------------------------------------------------------ */
/* Mode step, Sec. IV: Eq. (e10) integrated with the integrating factor of   */
/* Eq. (d3), noise of Eq. (d6), coupling integral of Eq. (f2), and the      */
/* shear drift of Eq. (btum).                                               */
/* ------------------------------------------------------------------------ */
void orc_step_modes(int M, int n_chains, const uint32_t *chain_id, double *R,
                    double nu, double T_star, double dtau, double gamma_dot,
                    int nonlinear, uint64_t seed, int64_t step0,
                    int64_t n_steps)
{
    double *phi = malloc(sizeof(double) * M * M);
    double *zl = malloc(sizeof(double) * M), *z = malloc(sizeof(double) * M);
    double *E = malloc(sizeof(double) * M), *C = malloc(sizeof(double) * M);
    double *W = malloc(sizeof(double) * M);
    orc_tables(M, nu, T_star, dtau, phi, zl, z, E, C, W);

#pragma omp parallel
    {
        double *r = malloc(sizeof(double) * 3 * M);
        double *g = malloc(sizeof(double) * 3 * M);
        double *F = malloc(sizeof(double) * 3 * M);
        double *dH = malloc(sizeof(double) * 3 * M);
#pragma omp for schedule(dynamic, 1)
        for (int c = 0; c < n_chains; ++c) {
            double *Rc = R + (size_t)c * 3 * M;
            for (int64_t k = step0; k < step0 + n_steps; ++k) {
                if (nonlinear) {
                    positions_from_modes(M, phi, Rc, 1, r);
                    delta_h_from_positions(M, phi, nu, r, g, F, dH);
                }
                for (int p = 0; p < M; ++p) {
                    double ry_old = Rc[1 * M + p];
                    for (int a = 0; a < 3; ++a) {
                        double eta = orc_normal(seed, (uint32_t)p, chain_id[c],
                                                k, (uint32_t)a, 0u);
                        double v = E[p] * Rc[a * M + p] + W[p] * eta;
                        if (nonlinear && p > 0) v += C[p] * dH[a * M + p];
                        Rc[a * M + p] = v;
                    }
                    Rc[0 * M + p] += gamma_dot * dtau * E[p] * ry_old;
                }
            }
        }
        free(r); free(g); free(F); free(dH);
    }
    free(phi); free(zl); free(z); free(E); free(C); free(W);
}

/* ------------------------------------------------------------------------ */
/* Bead-space Euler step of Eqs. (b3)-(b5) (the paper's default method),    */
/* with the shear drift of Eq. (btum).  pos is 3*M per chain.               */
/*   h_n = dH'/du_n = (|u_n| - 1) u_n/|u_n| - nu (u_{n-1} + u_{n+1}),        */
/*   -dH'/dr_n = h_{n+1} - h_n, with u_0 = u_M = 0 and h_0 = h_M = 0.       */
/* ------------------------------------------------------------------------ */
void orc_bead_force(int M, double nu, const double *pos, double *f)
{
    double *u = malloc(sizeof(double) * 3 * (M + 1));
    double *h = malloc(sizeof(double) * 3 * (M + 1));
    for (int a = 0; a < 3; ++a) {
        u[a * (M + 1) + 0] = 0.0;
        u[a * (M + 1) + M] = 0.0;
        for (int n = 1; n < M; ++n)
            u[a * (M + 1) + n] = pos[a * M + n] - pos[a * M + n - 1];
    }
    for (int n = 0; n <= M; ++n) {
        if (n == 0 || n == M) {
            for (int a = 0; a < 3; ++a) h[a * (M + 1) + n] = 0.0;
            continue;
        }
        double l2 = 0.0;
        for (int a = 0; a < 3; ++a) l2 += u[a * (M + 1) + n] * u[a * (M + 1) + n];
        double l = sqrt(l2);
        for (int a = 0; a < 3; ++a) {
            double un = u[a * (M + 1) + n];
            double nb = u[a * (M + 1) + n - 1] + u[a * (M + 1) + n + 1];
            h[a * (M + 1) + n] = (l - 1.0) * un / l - nu * nb;
        }
    }
    for (int a = 0; a < 3; ++a)
        for (int n = 0; n < M; ++n)
            f[a * M + n] = h[a * (M + 1) + n + 1] - h[a * (M + 1) + n];
    free(u);
    free(h);
}

void orc_step_euler(int M, int n_chains, const uint32_t *chain_id, double *pos,
                    double nu, double T_star, double dtau, double gamma_dot,
                    uint64_t seed, int64_t step0, int64_t n_steps)
{
    const double amp = sqrt(2.0 * T_star * dtau);
#pragma omp parallel
    {
        double *f = malloc(sizeof(double) * 3 * M);
#pragma omp for schedule(dynamic, 1)
        for (int c = 0; c < n_chains; ++c) {
            double *x = pos + (size_t)c * 3 * M;
            for (int64_t k = step0; k < step0 + n_steps; ++k) {
                orc_bead_force(M, nu, x, f);
                for (int n = 0; n < M; ++n) {
                    double y_old = x[1 * M + n];
                    for (int a = 0; a < 3; ++a) {
                        double eta = orc_normal(seed, (uint32_t)n, chain_id[c],
                                                k, (uint32_t)a, 1u);
                        x[a * M + n] += dtau * f[a * M + n] + amp * eta;
                    }
                    x[0 * M + n] += gamma_dot * dtau * y_old;
                }
            }
        }
        free(f);
    }
}

/* Reduced Hamiltonian H' = H/(lambda d^2) of Eq. (a2) times T*:
   H' = 1/2 sum_n (|u_n| - 1)^2 - nu sum_n u_n . u_{n+1}. */
double orc_energy(int M, double nu, const double *pos)
{
    double e = 0.0;
    double up[3] = {0, 0, 0};
    for (int n = 1; n < M; ++n) {
        double u[3], l2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            u[a] = pos[a * M + n] - pos[a * M + n - 1];
            l2 += u[a] * u[a];
        }
        double l = sqrt(l2);
        e += 0.5 * (l - 1.0) * (l - 1.0);
        if (n >= 2) e -= nu * (u[0] * up[0] + u[1] * up[1] + u[2] * up[2]);
        for (int a = 0; a < 3; ++a) up[a] = u[a];
    }
    return e;
}

/* ------------------------------------------------------------------------ */
/* The nu -> 0 limit (Sec. VI.A, Eqs. y2-y14): the inextensible wormlike      */
/* chain in the bending time scale tau-bar = nu tau, T-bar = T* / nu, with   */
/* Hamiltonian -sum_n u_n . u_{n+1} and bonds of unit length kept by the     */
/* tensions f_n.  One step of length dt moves bead n by                      */
/*   dr_n = (-f_n u_n + f_{n+1} u_{n+1} + h_{n+1} - h_n) dt                  */
/*          + sqrt(2 T-bar dt) eta_n                                         */
/* (Eq. y8) with h_n = -(u_{n-1} + u_{n+1}) the bending gradient on bond n;  */
/* tension and bending act along the midpoint bonds                          */
/* u^m_n = (u_n + u'_n)/|u_n + u'_n| (Eq. y14), and the f_n solve the        */
/* tridiagonal system that keeps |u'_n| = |u_n| (Eqs. y11-y13):              */
/*   (u_n + u'_n) . du_n = 0,                                                */
/*   du_n = (f_{n-1} u^m_{n-1} - 2 f_n u^m_n + f_{n+1} u^m_{n+1}) dt + D_n,   */
/* D_n the regular part of dr_n - dr_{n-1}.  Starting from u' = u the cycle  */
/* (midpoint, forces, tensions, u') is repeated until it converges: at most */
/* `iters` times, and with tol > 0 it stops after the first cycle that     */
/* changes no component of any u'_n by more than tol.  Bonds are            */
/* numbered n = 1..N (N = M - 1); f, h, u vanish outside.  Noise: the Euler  */
/* convention with tag 3.  pos is 3*M per chain; only the bonds and bead 0   */
/* are advanced, and the positions rebuilt from them.                       */
/* ------------------------------------------------------------------------ */
static void wlc_solve(int N, const double *a, const double *b, const double *c,
                      const double *r, double *x, double *cp, double *dp)
{
    /* Thomas algorithm: a_n x_{n-1} + b_n x_n + c_n x_{n+1} = r_n, n < N */
    cp[0] = c[0] / b[0];
    dp[0] = r[0] / b[0];
    for (int n = 1; n < N; ++n) {
        const double m = b[n] - a[n] * cp[n - 1];
        cp[n] = c[n] / m;
        dp[n] = (r[n] - a[n] * dp[n - 1]) / m;
    }
    x[N - 1] = dp[N - 1];
    for (int n = N - 2; n >= 0; --n) x[n] = dp[n] - cp[n] * x[n + 1];
}

void orc_step_wlc(int M, int n_chains, const uint32_t *chain_id, double *pos,
                  double T_bar, double dt, int iters, double tol, int midpoint,
                  uint64_t seed, int64_t step0, int64_t n_steps)
{
    const int N = M - 1;
    const double amp = sqrt(2.0 * T_bar * dt);
#pragma omp parallel
    {
        /* bonds u[n][a], n = 0..N+1 with u[0] = u[N+1] = 0 (bond n = 1..N) */
        double *u = calloc((size_t)3 * (N + 2), sizeof(double));
        double *un = calloc((size_t)3 * (N + 2), sizeof(double));
        double *um = calloc((size_t)3 * (N + 2), sizeof(double));
        double *w = calloc((size_t)3 * (N + 2), sizeof(double));
        double *h = calloc((size_t)3 * (N + 2), sizeof(double));
        double *dr = calloc((size_t)3 * (N + 1), sizeof(double));
        double *eta = calloc((size_t)3 * (N + 1), sizeof(double));
        double *D = calloc((size_t)3 * (N + 2), sizeof(double));
        double *f = calloc((size_t)(N + 2), sizeof(double));
        double *A = malloc(sizeof(double) * N), *Bd = malloc(sizeof(double) * N);
        double *Cd = malloc(sizeof(double) * N), *Rr = malloc(sizeof(double) * N);
        double *X = malloc(sizeof(double) * N), *cp = malloc(sizeof(double) * N);
        double *dp = malloc(sizeof(double) * N);
#pragma omp for schedule(dynamic, 1)
        for (int c = 0; c < n_chains; ++c) {
            double *x = pos + (size_t)c * 3 * M;
            for (int n = 1; n <= N; ++n)
                for (int a = 0; a < 3; ++a) u[3 * n + a] = x[a * M + n] - x[a * M + n - 1];
            double r0[3] = {x[0], x[M], x[2 * M]};
            for (int64_t k = step0; k < step0 + n_steps; ++k) {
                for (int a = 0; a < 3; ++a)
                    for (int n = 0; n <= N; ++n)
                        eta[3 * n + a] = orc_normal(seed, (uint32_t)n, chain_id[c], k,
                                                    (uint32_t)a, 3u);
                memcpy(un, u, sizeof(double) * 3 * (N + 2));
                for (int it = 0; it < iters; ++it) {
                    /* midpoint bonds and the constraint weights */
                    for (int n = 1; n <= N; ++n) {
                        double s2 = 0.0;
                        for (int a = 0; a < 3; ++a) {
                            w[3 * n + a] = u[3 * n + a] + un[3 * n + a];
                            s2 += w[3 * n + a] * w[3 * n + a];
                        }
                        /* Eq. (y14); or, with midpoint == 0, the bond at the
                           start of the step (forces as first written in y8, y9) */
                        for (int a = 0; a < 3; ++a)
                            um[3 * n + a] = midpoint ? w[3 * n + a] / sqrt(s2) : u[3 * n + a];
                    }
                    /* bending gradient on each bond, at the midpoint */
                    for (int n = 1; n <= N; ++n)
                        for (int a = 0; a < 3; ++a)
                            h[3 * n + a] = -(um[3 * (n - 1) + a] + um[3 * (n + 1) + a]);
                    /* regular bead displacements and their bond differences */
                    for (int n = 0; n <= N; ++n)
                        for (int a = 0; a < 3; ++a) {
                            const double hn = n >= 1 ? h[3 * n + a] : 0.0;
                            const double hn1 = n + 1 <= N ? h[3 * (n + 1) + a] : 0.0;
                            dr[3 * n + a] = (hn1 - hn) * dt + amp * eta[3 * n + a];
                        }
                    for (int n = 1; n <= N; ++n)
                        for (int a = 0; a < 3; ++a)
                            D[3 * n + a] = dr[3 * n + a] - dr[3 * (n - 1) + a];
                    /* tensions: w_n . (f_{n-1} um_{n-1} - 2 f_n um_n + f_{n+1} um_{n+1}) dt
                       = -w_n . D_n */
                    for (int n = 1; n <= N; ++n) {
                        double wl = 0.0, wm = 0.0, wr = 0.0, wd = 0.0;
                        for (int a = 0; a < 3; ++a) {
                            wl += w[3 * n + a] * um[3 * (n - 1) + a];
                            wm += w[3 * n + a] * um[3 * n + a];
                            wr += w[3 * n + a] * um[3 * (n + 1) + a];
                            wd += w[3 * n + a] * D[3 * n + a];
                        }
                        A[n - 1] = wl * dt;
                        Bd[n - 1] = -2.0 * wm * dt;
                        Cd[n - 1] = wr * dt;
                        Rr[n - 1] = -wd;
                    }
                    wlc_solve(N, A, Bd, Cd, Rr, X, cp, dp);
                    f[0] = f[N + 1] = 0.0;
                    for (int n = 1; n <= N; ++n) f[n] = X[n - 1];
                    double change = 0.0;
                    for (int n = 1; n <= N; ++n)
                        for (int a = 0; a < 3; ++a) {
                            const double v = u[3 * n + a] + D[3 * n + a] +
                                             (f[n - 1] * um[3 * (n - 1) + a] -
                                              2.0 * f[n] * um[3 * n + a] +
                                              f[n + 1] * um[3 * (n + 1) + a]) * dt;
                            change = fmax(change, fabs(v - un[3 * n + a]));
                            un[3 * n + a] = v;
                        }
                    if (tol > 0.0 && change <= tol) break;
                }
                /* bead 0 moves with its own tension, bending and noise */
                for (int a = 0; a < 3; ++a)
                    r0[a] += dr[a] + (N >= 1 ? f[1] * um[3 + a] * dt : 0.0);
                memcpy(u, un, sizeof(double) * 3 * (N + 2));
            }
            for (int a = 0; a < 3; ++a) {
                x[a * M] = r0[a];
                for (int n = 1; n <= N; ++n) x[a * M + n] = x[a * M + n - 1] + u[3 * n + a];
            }
        }
        free(u); free(un); free(um); free(w); free(h); free(dr); free(eta); free(D);
        free(f); free(A); free(Bd); free(Cd); free(Rr); free(X); free(cp); free(dp);
    }
}

/* ------------------------------------------------------------------------ */
/* Metropolis Monte Carlo in the mode representation, the paper's           */
/* equilibrium benchmark (Sec. V.B: "large MC steps in the slow modes and     */
/* small steps in the fast modes").  The paper gives no more detail; this   */
/* is the reading used.  One sweep proposes, for p = 1..M-1 and component   */
/* a = x, y, z in that order, R_p^a -> R_p^a + delta with delta uniform on  */
/* (-s_p, s_p), s_p = scale * sqrt(T* / zeta^l_p) (the width of mode p      */
/* under the harmonic Hamiltonian of Eqs. c6, c9), and accepts it with      */
/* probability min(1, exp(-(H'_new - H'_old) / T*)), H' of Eq. (b3) on the  */
/* positions.  Random numbers: the Philox block of counter (p, chain,       */
/* step = sweep index, component a, tag 2); word 0 gives delta =            */
/* s_p (2 U0 - 1), word 1 the uniform U1 of the test U1 < exp(-dH'/T*),    */
/* U = (x + 1/2) 2^-32.  The centre of mass does not enter H' and is left   */
/* unchanged.  accepted[c] receives the number of accepted proposals.      */
/* ------------------------------------------------------------------------ */
void orc_mc_sweeps(int M, int n_chains, const uint32_t *chain_id, double *R,
                   double nu, double T_star, double scale, uint64_t seed,
                   int64_t step0, int64_t n_sweeps, int64_t *accepted)
{
    double *phi = malloc(sizeof(double) * M * M);
    double *zl = malloc(sizeof(double) * M), *z = malloc(sizeof(double) * M);
    double *E = malloc(sizeof(double) * M), *C = malloc(sizeof(double) * M);
    double *W = malloc(sizeof(double) * M);
    orc_tables(M, nu, T_star, 1.0, phi, zl, z, E, C, W);
    const double two_m32 = 1.0 / 4294967296.0;
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};

#pragma omp parallel
    {
        double *r = malloc(sizeof(double) * 3 * M);
        double *rt = malloc(sizeof(double) * 3 * M);
#pragma omp for schedule(dynamic, 1)
        for (int c = 0; c < n_chains; ++c) {
            double *Rc = R + (size_t)c * 3 * M;
            int64_t acc = 0;
            positions_from_modes(M, phi, Rc, 0, r);
            double e = orc_energy(M, nu, r);
            for (int64_t k = step0; k < step0 + n_sweeps; ++k) {
                const uint64_t ku = (uint64_t)k;
                for (int p = 1; p < M; ++p) {
                    const double sp = scale * sqrt(T_star / zl[p]);
                    for (int a = 0; a < 3; ++a) {
                        uint32_t ctr[4] = {(uint32_t)p, chain_id[c], (uint32_t)ku,
                                           (uint32_t)((ku >> 32) << 8) |
                                               ((uint32_t)a << 4) | 2u};
                        uint32_t x[4];
                        orc_philox4x32_10(ctr, key, x);
                        const double u0 = ((double)x[0] + 0.5) * two_m32;
                        const double u1 = ((double)x[1] + 0.5) * two_m32;
                        const double delta = sp * (2.0 * u0 - 1.0);
                        memcpy(rt, r, sizeof(double) * 3 * M);
                        for (int n = 0; n < M; ++n)
                            rt[a * M + n] += phi[n * M + p] * delta;
                        const double et = orc_energy(M, nu, rt);
                        if (u1 < exp(-(et - e) / T_star)) {
                            memcpy(r, rt, sizeof(double) * 3 * M);
                            Rc[a * M + p] += delta;
                            e = et;
                            ++acc;
                        }
                    }
                }
            }
            accepted[c] = acc;
        }
        free(r); free(rt);
    }
    free(phi); free(zl); free(z); free(E); free(C); free(W);
}

/* ------------------------------------------------------------------------ */
/* Observables of Sec. V.B: per chain, from positions (3*M).                 */
/* out[0] mean bond length, out[1] |L|^2 with L = r_{M-1} - r_0,            */
/* out[2..4] L, out[5..7] centre of mass, out[8..10] middle bond            */
/* u_m (m = M/2), out[11..13] r_mid - r_cm (mid = (M-1)/2),                 */
/* out[14] x extent max x - min x, out[15] mean squared bond length.        */
/* ------------------------------------------------------------------------ */
void orc_chain_observables(int M, const double *pos, double *out)
{
    double lsum = 0.0, l2sum = 0.0;
    for (int n = 1; n < M; ++n) {
        double l2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            double u = pos[a * M + n] - pos[a * M + n - 1];
            l2 += u * u;
        }
        lsum += sqrt(l2);
        l2sum += l2;
    }
    out[0] = lsum / (M - 1);
    double L[3], cm[3];
    for (int a = 0; a < 3; ++a) {
        L[a] = pos[a * M + M - 1] - pos[a * M + 0];
        double s = 0.0;
        for (int n = 0; n < M; ++n) s += pos[a * M + n];
        cm[a] = s / M;
    }
    out[1] = L[0] * L[0] + L[1] * L[1] + L[2] * L[2];
    int m = M / 2, mid = (M - 1) / 2;
    for (int a = 0; a < 3; ++a) {
        out[2 + a] = L[a];
        out[5 + a] = cm[a];
        out[8 + a] = pos[a * M + m] - pos[a * M + m - 1];
        out[11 + a] = pos[a * M + mid] - cm[a];
    }
    double xmin = pos[0], xmax = pos[0];
    for (int n = 1; n < M; ++n) {
        if (pos[n] < xmin) xmin = pos[n];
        if (pos[n] > xmax) xmax = pos[n];
    }
    out[14] = xmax - xmin;
    out[15] = l2sum / (M - 1);
}
