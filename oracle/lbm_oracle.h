/*
 * Plain FP64 CPU oracle of the binary free-energy lattice Boltzmann method of
 * Pooley, Kusumaatmaja and Yeomans, "Contact line dynamics in binary lattice
 * Boltzmann simulations" (arXiv:0812.1282).
 *
 * TEST INFRASTRUCTURE. This code exists only to check the HIP library. It is
 * built, linked and run by the tests, by the smoke check and by the CPU
 * baseline leg of the benchmark, never by the product path. It shares no code,
 * header, table or helper with the HIP library.
 *
 * Every routine follows the paper step by step on whole fields, in double
 * precision, with the paper's matrices written out as printed:
 *   moments                      Sec. III.A, Eq. (moments)
 *   chemical potential, p0       Sec. II, Eqs. (chempot), (p0)
 *   equilibria, stencils         Appendix A, Eqs. (equilibrium), (feq0), (best)
 *   BGK collision                Sec. III.A, Eqs. (latbolt), (gevo)
 *   MRT collision                Sec. III.B, Eqs. (mrtlb), (Matrix), (diag)
 *   phi-dependent tau            Sec. IV, Eq. (tau)
 *   streaming, bounce-back       Sec. III.A, Eqs. (stream1), (stream2); Sec. V.B
 *   the four-step MRT algorithm  Sec. VI (Steps 1-4)
 *
 * Layout: node (x, y) has index y*nx + x; a population plane i is the block
 * [i*nx*ny, (i+1)*nx*ny). The lattice is doubly periodic; walls are solid
 * nodes of the mask (mid-link bounce-back between a fluid and a solid node).
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t nx, ny;
    double A, B;          /* mu = A phi + B phi^3 - kappa lap phi (paper: A = -a, B = a) */
    double kappa, Gamma;
    double tau_alpha;     /* tau at phi = +1 */
    double tau_beta;      /* tau at phi = -1 */
    double tau_phi;
    int32_t collision;    /* 0 = BGK, 1 = MRT */
    int32_t zero_u_feq;   /* Step 2: u = 0 at boundary nodes in f^eq */
    int32_t zero_u_geq;   /* Step 2 applied to g^eq as well */
    int32_t tau_clamp;    /* 1: phi clamped to [-1, 1] inside Eq. (tau); 0: the law as printed */
    int32_t tau_lut;      /* >= 2: tau taken from a table of this many values (Sec. VI);
                             0: Eq. (tau) itself */
    int32_t bounce;       /* 0: mid-link bounce-back (Fig. 9a); 1: lattice-node
                             bounce-back (Fig. 9b), the wall on the boundary nodes */
} orc_params;

typedef struct orc_state orc_state;

/* Create a lattice whose state S_0 is the equilibrium of the given fields.
 * solid: nx*ny (nonzero = solid). dphi: nx*ny wall gradient d_perp phi at
 * solid nodes (NULL = 0). phi0 required; rho0 (NULL = 1), ux0, uy0 (NULL = 0).
 * Returns NULL on invalid arguments. */
orc_state* orc_create(const orc_params* p, const uint8_t* solid, const double* dphi,
                      const double* phi0, const double* rho0, const double* ux0,
                      const double* uy0);
void orc_free(orc_state* s);
void orc_step(orc_state* s, int64_t nsteps);
int64_t orc_step_count(const orc_state* s);
void orc_set_wall_dphi(orc_state* s, const double* dphi);

/* Moments of the current state S_n (zero at solid nodes); any pointer may be NULL. */
void orc_fields(const orc_state* s, double* phi, double* rho, double* ux, double* uy);
/* Copy S_n out (9*nx*ny each) or overwrite it. */
void orc_get_populations(const orc_state* s, double* f, double* g);
void orc_set_populations(orc_state* s, const double* f, const double* g);
/* Compensated sums over fluid nodes: out[0]=sum rho, out[1]=sum phi,
 * out[2]=sum rho|u|^2/2, out[3]=max |u|, out[4]=number of fluid nodes. */
void orc_diagnostics(const orc_state* s, double out[5]);

/* ---- the individual steps, exposed for the pins ---- */
void orc_lattice(int32_t ex[9], int32_t ey[9], double w[9], double wxx[9], double wyy[9],
                 double wxy[9]);
void orc_mrt_matrices(double M[81], double Minv[81]);
void orc_moments(int32_t nx, int32_t ny, const uint8_t* solid, const double* f,
                 const double* g, double* rho, double* phi, double* ux, double* uy);
void orc_ghosts(int32_t nx, int32_t ny, const uint8_t* solid, const double* dphi,
                const double* phi, double* phix);
void orc_gradients(int32_t nx, int32_t ny, const uint8_t* solid, const double* phix,
                   double* dx, double* dy, double* lap);
void orc_equilibria_node(const orc_params* p, double rho, double phi, double ux, double uy,
                         double ux_f, double uy_f, double dxphi, double dyphi,
                         double lapphi, double feq[9], double geq[9]);
void orc_collide_node(const orc_params* p, double phi, const double f[9],
                      const double feq[9], const double g[9], const double geq[9],
                      double fpost[9], double gpost[9]);
void orc_stream(int32_t nx, int32_t ny, const uint8_t* solid, const double* post,
                double* next);
void orc_stream_lattice_node(int32_t nx, int32_t ny, const uint8_t* solid, const double* post,
                             double* next);
void orc_reflect_walls(int32_t nx, int32_t ny, const uint8_t* solid, const double* pre,
                       double* post);
double orc_tau(const orc_params* p, double phi);

void orc_set_threads(int32_t n);
int32_t orc_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif
