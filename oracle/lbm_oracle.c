/*
 * Plain FP64 CPU oracle of the binary free-energy lattice Boltzmann method of
 * Pooley, Kusumaatmaja and Yeomans (arXiv:0812.1282).
 *
 * TEST INFRASTRUCTURE. Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark build, load or run this file. It shares no code with
 * the HIP library.
 *
 * The oracle is the algorithm itself, written on whole fields with plain
 * loops, in the order of the paper's four-step procedure (Sec. VI):
 *   Step 1  moments                         Eq. (moments)
 *           ghost phi at wetting walls      Sec. II (d_perp phi = xi/kappa), Sec. IV
 *           stencils for grad and laplacian Appendix A, Eq. (best)
 *           mu and p0                       Eqs. (chempot), (p0)
 *           tau(phi)                        Eq. (tau)
 *   Step 2  u = 0 at boundary nodes in the equilibrium (flag)
 *           equilibria                      Appendix A, Eqs. (equilibrium), (feq0)
 *   Step 3  collision: BGK Eqs. (latbolt), (gevo) or MRT Eqs. (mrtlb), (Matrix), (diag)
 *   Step 4  streaming with mid-link bounce-back, Eqs. (stream1), (stream2), Sec. V.B
 *
 * Readings of points the paper leaves open (shared with the HIP library only
 * through their description, never through code):
 *  - d_perp points from the wall into the fluid; the gradient is imposed
 *    through a ghost value of phi at each solid node next to the fluid: the
 *    mean of phi over its fluid axis neighbours minus d_perp phi (a central
 *    difference across the mid-link wall plane). A solid node whose only fluid
 *    neighbours are diagonal uses the mean over those minus sqrt(2) d_perp phi.
 *  - a boundary node is a fluid node with at least one solid node among its
 *    eight lattice neighbours.
 *  - tau(phi) is the linear law of Eq. (tau) in the node's current phi, with
 *    no clamp; both bulk values must exceed 1/2. An option (tau_clamp) clamps
 *    phi to [-1, 1] first, for runs where phi overshoots a bulk value whose
 *    tau is close to 1/2.
 *  - bounce-back applies to g as well as to f.
 *  - lattice-node bounce-back (Fig. 9b, option): a wall node is a solid node
 *    with a fluid node among its eight neighbours. It holds the populations
 *    that streamed into it and, in place of a collision, reverses them, so a
 *    population sent into the wall returns to the node it left two steps
 *    later (one with mid-link). At S_0 a wall node holds what its fluid
 *    neighbours' equilibria send into it; populations between wall nodes stay
 *    zero. Mass is then conserved over fluid and wall nodes together.
 *  - the tau table of Sec. VI (option): tau_lut values of tau evenly spaced
 *    from tau_beta to tau_alpha (viscosity is linear in tau, so the spacing is
 *    even in viscosity too); a node takes the entry closest to its Eq. (tau)
 *    value, the lower-index entry on a tie, which also limits tau to the
 *    bulk range.
 *  - the stencil for d/dy is the printed d/dx stencil rotated by 90 degrees.
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Lattice vectors, Sec. III.A: e0 = 0, e1,2 = (+-1, 0), e3,4 = (0, +-1),
 * e5,6 = (+-1, +-1), e7,8 = (-+1, +-1). */
static const int EX[9] = {0, 1, -1, 0, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 0, 1, -1, 1, -1, 1, -1};

/* Equilibrium weights, Appendix A. */
static const double W[9] = {0.0, 1.0 / 3, 1.0 / 3, 1.0 / 3, 1.0 / 3,
                            1.0 / 12, 1.0 / 12, 1.0 / 12, 1.0 / 12};
static const double WXX[9] = {0.0, 1.0 / 3, 1.0 / 3, -1.0 / 6, -1.0 / 6,
                              -1.0 / 24, -1.0 / 24, -1.0 / 24, -1.0 / 24};
static const double WYY[9] = {0.0, -1.0 / 6, -1.0 / 6, 1.0 / 3, 1.0 / 3,
                              -1.0 / 24, -1.0 / 24, -1.0 / 24, -1.0 / 24};
static const double WXY[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.25, 0.25, -0.25, -0.25};

/* Transform matrix of the MRT collision, Eq. (Matrix), typed as printed. */
static const double MRT_M[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, -1, 0, 0, 1, -1, -1, 1},
    {0, -2, 2, 0, 0, 1, -1, -1, 1},
    {0, 0, 0, 1, -1, 1, -1, 1, -1},
    {0, 0, 0, -2, 2, 1, -1, 1, -1},
    {0, 1, 1, -1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, 1, -1, -1},
};

/* Stencils of Eq. (best). Matrix row 0 is the row above the node (y+1), row 2
 * the row below (y-1); column 0 is x-1, column 2 is x+1. */
static const double STENCIL_DX[3][3] = {{-1, 0, 1}, {-4, 0, 4}, {-1, 0, 1}};  /* / 12 */
static const double STENCIL_DY[3][3] = {{1, 4, 1}, {0, 0, 0}, {-1, -4, -1}};  /* / 12 */
static const double STENCIL_LAP[3][3] = {{1, 4, 1}, {4, -20, 4}, {1, 4, 1}};  /* / 6 */

struct orc_state {
    orc_params p;
    int64_t step;
    size_t n;
    uint8_t* solid;
    uint8_t* boundary;
    double* dphi;
    double* f;
    double* g;
    /* per-step fields */
    double *rho, *phi, *ux, *uy, *phix, *dx, *dy, *lap;
    double *fpost, *gpost;
};

static inline int wrap(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

void orc_lattice(int32_t ex[9], int32_t ey[9], double w[9], double wxx[9], double wyy[9],
                 double wxy[9]) {
    for (int i = 0; i < 9; ++i) {
        if (ex) ex[i] = EX[i];
        if (ey) ey[i] = EY[i];
        if (w) w[i] = W[i];
        if (wxx) wxx[i] = WXX[i];
        if (wyy) wyy[i] = WYY[i];
        if (wxy) wxy[i] = WXY[i];
    }
}

/* M^-1_ij = M_ji / sum_k M_jk^2, Sec. III.B. */
void orc_mrt_matrices(double M[81], double Minv[81]) {
    for (int i = 0; i < 9; ++i)
        for (int j = 0; j < 9; ++j) {
            if (M) M[i * 9 + j] = MRT_M[i][j];
            if (Minv) {
                double norm = 0.0;
                for (int k = 0; k < 9; ++k) norm += MRT_M[j][k] * MRT_M[j][k];
                Minv[i * 9 + j] = MRT_M[j][i] / norm;
            }
        }
}

/* Eq. (moments): rho = sum f, phi = sum g, rho v = sum f e. */
void orc_moments(int32_t nx, int32_t ny, const uint8_t* solid, const double* f,
                 const double* g, double* rho, double* phi, double* ux, double* uy) {
    const size_t n = (size_t)nx * ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const size_t r = (size_t)y * nx + x;
            double sr = 0.0, sp = 0.0, jx = 0.0, jy = 0.0;
            if (!solid[r]) {
                for (int i = 0; i < 9; ++i) {
                    sr += f[i * n + r];
                    sp += g[i * n + r];
                    jx += f[i * n + r] * EX[i];
                    jy += f[i * n + r] * EY[i];
                }
            }
            if (rho) rho[r] = sr;
            if (phi) phi[r] = sp;
            if (ux) ux[r] = solid[r] ? 0.0 : jx / sr;
            if (uy) uy[r] = solid[r] ? 0.0 : jy / sr;
        }
}

/* phi with ghost values at solid nodes (the wetting condition d_perp phi = xi/kappa). */
void orc_ghosts(int32_t nx, int32_t ny, const uint8_t* solid, const double* dphi,
                const double* phi, double* phix) {
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const size_t r = (size_t)y * nx + x;
            if (!solid[r]) {
                phix[r] = phi[r];
                continue;
            }
            double sum_axis = 0.0, sum_diag = 0.0;
            int n_axis = 0, n_diag = 0;
            for (int k = 1; k < 9; ++k) {
                const size_t q = (size_t)wrap(y + EY[k], ny) * nx + wrap(x + EX[k], nx);
                if (solid[q]) continue;
                if (k <= 4) {
                    sum_axis += phi[q];
                    ++n_axis;
                } else {
                    sum_diag += phi[q];
                    ++n_diag;
                }
            }
            const double grad = dphi ? dphi[r] : 0.0;
            if (n_axis > 0)
                phix[r] = sum_axis / n_axis - grad;
            else if (n_diag > 0)
                phix[r] = sum_diag / n_diag - sqrt(2.0) * grad;
            else
                phix[r] = 0.0;
        }
}

/* Eq. (best) applied at every fluid node to phi-with-ghosts. */
void orc_gradients(int32_t nx, int32_t ny, const uint8_t* solid, const double* phix,
                   double* dx, double* dy, double* lap) {
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const size_t r = (size_t)y * nx + x;
            double sx = 0.0, sy = 0.0, sl = 0.0;
            if (!solid || !solid[r]) {
                for (int row = 0; row < 3; ++row)
                    for (int col = 0; col < 3; ++col) {
                        const int yy = wrap(y + 1 - row, ny);
                        const int xx = wrap(x - 1 + col, nx);
                        const double v = phix[(size_t)yy * nx + xx];
                        sx += STENCIL_DX[row][col] * v;
                        sy += STENCIL_DY[row][col] * v;
                        sl += STENCIL_LAP[row][col] * v;
                    }
                sx /= 12.0;
                sy /= 12.0;
                sl /= 6.0;
            }
            if (dx) dx[r] = sx;
            if (dy) dy[r] = sy;
            if (lap) lap[r] = sl;
        }
}

/* Eq. (tau): linear in the node's phi; with tau_clamp, phi is first limited to
 * the bulk range [-1, 1]. */
static double lut_entry(const orc_params* p, int k) {
    return p->tau_beta + k * ((p->tau_alpha - p->tau_beta) / (p->tau_lut - 1));
}

double orc_tau(const orc_params* p, double phi) {
    if (p->tau_clamp) phi = phi > 1.0 ? 1.0 : (phi < -1.0 ? -1.0 : phi);
    const double tau = p->tau_beta + 0.5 * (phi + 1.0) * (p->tau_alpha - p->tau_beta);
    if (p->tau_lut < 2) return tau;
    /* Sec. VI: the closest entry of the table. The entries run monotonically
     * from tau_beta to tau_alpha; bisect for the last one not past tau, then
     * take it or the next, whichever is closer (the first on a tie). */
    const double dir = p->tau_alpha >= p->tau_beta ? 1.0 : -1.0;
    int lo = 0, hi = p->tau_lut - 1;
    if (dir * (lut_entry(p, lo) - tau) >= 0.0) return lut_entry(p, lo);
    if (dir * (lut_entry(p, hi) - tau) <= 0.0) return lut_entry(p, hi);
    while (hi - lo > 1) {
        const int mid = lo + (hi - lo) / 2;
        if (dir * (lut_entry(p, mid) - tau) <= 0.0)
            lo = mid;
        else
            hi = mid;
    }
    return fabs(lut_entry(p, hi) - tau) < fabs(tau - lut_entry(p, lo)) ? lut_entry(p, hi)
                                                                        : lut_entry(p, lo);
}

/* Appendix A, Eqs. (equilibrium) and (feq0), with c = 1, and Eqs. (chempot), (p0)
 * for mu and p0. (ux_f, uy_f) is the velocity used in f^eq (zero at boundary
 * nodes under Step 2); (ux, uy) is the velocity used in g^eq. */
void orc_equilibria_node(const orc_params* p, double rho, double phi, double ux, double uy,
                         double ux_f, double uy_f, double dxphi, double dyphi,
                         double lapphi, double feq[9], double geq[9]) {
    const double p0 = rho / 3.0 + p->A * phi * phi / 2.0 + 3.0 * p->B * phi * phi * phi * phi / 4.0;
    const double mu = p->A * phi + p->B * phi * phi * phi - p->kappa * lapphi;
    const double uf[2] = {ux_f, uy_f};
    const double ug[2] = {ux, uy};
    double fsum = 0.0, gsum = 0.0;
    for (int i = 1; i < 9; ++i) {
        const double e[2] = {(double)EX[i], (double)EY[i]};
        double eu_f = 0.0, eu_g = 0.0, quad_f = 0.0, quad_g = 0.0;
        for (int a = 0; a < 2; ++a) {
            eu_f += e[a] * uf[a];
            eu_g += e[a] * ug[a];
            for (int b = 0; b < 2; ++b) {
                const double t = e[a] * e[b] - (a == b ? 1.0 / 3.0 : 0.0);
                quad_f += t * uf[a] * uf[b];
                quad_g += t * ug[a] * ug[b];
            }
        }
        feq[i] = W[i] * (p0 - p->kappa * phi * lapphi + rho * eu_f + 1.5 * rho * quad_f) +
                 p->kappa * (WXX[i] * dxphi * dxphi + WYY[i] * dyphi * dyphi +
                             WXY[i] * dxphi * dyphi);
        geq[i] = W[i] * (p->Gamma * mu + phi * eu_g + 1.5 * phi * quad_g);
        fsum += feq[i];
        gsum += geq[i];
    }
    feq[0] = rho - fsum;
    geq[0] = phi - gsum;
}

/* Collision: BGK Eq. (latbolt) or MRT Eq. (mrtlb) with S of Eq. (diag) and
 * omega = 1/tau(phi); g always relaxes with Eq. (gevo). */
void orc_collide_node(const orc_params* p, double phi, const double f[9],
                      const double feq[9], const double g[9], const double geq[9],
                      double fpost[9], double gpost[9]) {
    const double tau = orc_tau(p, phi);
    if (p->collision == 0) {
        for (int i = 0; i < 9; ++i) fpost[i] = f[i] - (f[i] - feq[i]) / tau;
    } else {
        double Minv[81];
        orc_mrt_matrices(NULL, Minv);
        const double omega = 1.0 / tau;
        const double S[9] = {0, 1, 1, 0, 1, 0, 1, omega, omega};
        double d[9], m[9];
        for (int i = 0; i < 9; ++i) d[i] = f[i] - feq[i];
        for (int j = 0; j < 9; ++j) {
            m[j] = 0.0;
            for (int i = 0; i < 9; ++i) m[j] += MRT_M[j][i] * d[i];
            m[j] *= S[j];
        }
        for (int i = 0; i < 9; ++i) {
            double c = 0.0;
            for (int j = 0; j < 9; ++j) c += Minv[i * 9 + j] * m[j];
            fpost[i] = f[i] - c;
        }
    }
    for (int i = 0; i < 9; ++i) gpost[i] = g[i] - (g[i] - geq[i]) / p->tau_phi;
}

/* Eqs. (stream1)/(stream2) with mid-link bounce-back: a post-collision
 * population moving from fluid node r along e_i lands on r + e_i when that node
 * is fluid, otherwise it returns to r in the opposite direction. */
void orc_stream(int32_t nx, int32_t ny, const uint8_t* solid, const double* post,
                double* next) {
    static const int OPP[9] = {0, 2, 1, 4, 3, 6, 5, 8, 7};
    const size_t n = (size_t)nx * ny;
    memset(next, 0, 9 * n * sizeof(double));
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const size_t r = (size_t)y * nx + x;
            if (solid[r]) continue;
            for (int i = 0; i < 9; ++i) {
                const size_t q = (size_t)wrap(y + EY[i], ny) * nx + wrap(x + EX[i], nx);
                if (!solid[q])
                    next[i * n + q] = post[i * n + r];
                else
                    next[OPP[i] * n + r] = post[i * n + r];
            }
        }
}

/* A solid node with a fluid node among its eight neighbours. */
static int is_wall(int32_t nx, int32_t ny, const uint8_t* solid, int x, int y) {
    if (!solid[(size_t)y * nx + x]) return 0;
    for (int k = 1; k < 9; ++k)
        if (!solid[(size_t)wrap(y + EY[k], ny) * nx + wrap(x + EX[k], nx)]) return 1;
    return 0;
}

/* Lattice-node bounce-back, the wall nodes' part: each reverses the
 * populations it holds (post_i = pre_opp(i)) in place of a collision. */
void orc_reflect_walls(int32_t nx, int32_t ny, const uint8_t* solid, const double* pre,
                       double* post) {
    static const int OPP[9] = {0, 2, 1, 4, 3, 6, 5, 8, 7};
    const size_t n = (size_t)nx * ny;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            if (!is_wall(nx, ny, solid, x, y)) continue;
            const size_t r = (size_t)y * nx + x;
            for (int i = 0; i < 9; ++i) post[OPP[i] * n + r] = pre[i * n + r];
        }
}

/* Eqs. (stream1)/(stream2) with lattice-node bounce-back: every population of
 * a fluid or wall node moves along e_i to the next node; one that would enter
 * the interior of a solid (only a wall node can send it there) is dropped. */
void orc_stream_lattice_node(int32_t nx, int32_t ny, const uint8_t* solid, const double* post,
                             double* next) {
    const size_t n = (size_t)nx * ny;
    memset(next, 0, 9 * n * sizeof(double));
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const size_t r = (size_t)y * nx + x;
            if (solid[r] && !is_wall(nx, ny, solid, x, y)) continue;
            for (int i = 0; i < 9; ++i) {
                const int qx = wrap(x + EX[i], nx), qy = wrap(y + EY[i], ny);
                const size_t q = (size_t)qy * nx + qx;
                if (!solid[q] || is_wall(nx, ny, solid, qx, qy)) next[i * n + q] = post[i * n + r];
            }
        }
}

static int all_finite(const double* a, size_t n) {
    if (!a) return 1;
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

/* Equilibria of the current (rho, phi, u) fields into (f, g); apply_step2
 * selects Step 2 (u = 0 at boundary nodes) for f^eq and/or g^eq per the flags. */
static void equilibria_field(orc_state* s, int apply_step2, double* fout, double* gout) {
    const orc_params* p = &s->p;
    const int nx = p->nx, ny = p->ny;
    const size_t n = s->n;
    orc_ghosts(nx, ny, s->solid, s->dphi, s->phi, s->phix);
    orc_gradients(nx, ny, s->solid, s->phix, s->dx, s->dy, s->lap);
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const size_t r = (size_t)y * nx + x;
            if (s->solid[r]) continue;
            const int zf = apply_step2 && p->zero_u_feq && s->boundary[r];
            const int zg = apply_step2 && p->zero_u_geq && s->boundary[r];
            double feq[9], geq[9];
            orc_equilibria_node(p, s->rho[r], s->phi[r], zg ? 0.0 : s->ux[r],
                                zg ? 0.0 : s->uy[r], zf ? 0.0 : s->ux[r], zf ? 0.0 : s->uy[r],
                                s->dx[r], s->dy[r], s->lap[r], feq, geq);
            for (int i = 0; i < 9; ++i) {
                fout[i * n + r] = feq[i];
                gout[i * n + r] = geq[i];
            }
        }
}

orc_state* orc_create(const orc_params* p, const uint8_t* solid, const double* dphi,
                      const double* phi0, const double* rho0, const double* ux0,
                      const double* uy0) {
    if (!p || !solid || !phi0 || p->nx < 3 || p->ny < 3) return NULL;
    if (!(p->tau_alpha > 0.5) || !(p->tau_beta > 0.5) || !(p->tau_phi > 0.5)) return NULL;
    if ((p->bounce != 0 && p->bounce != 1) || p->tau_lut < 0 || p->tau_lut == 1) return NULL;
    const size_t n = (size_t)p->nx * p->ny;
    if (!all_finite(phi0, n) || !all_finite(rho0, n) || !all_finite(ux0, n) ||
        !all_finite(uy0, n) || !all_finite(dphi, n))
        return NULL;
    orc_state* s = (orc_state*)calloc(1, sizeof(orc_state));
    s->p = *p;
    s->n = n;
    s->solid = (uint8_t*)malloc(n);
    s->boundary = (uint8_t*)calloc(n, 1);
    s->dphi = (double*)calloc(n, sizeof(double));
    s->f = (double*)calloc(9 * n, sizeof(double));
    s->g = (double*)calloc(9 * n, sizeof(double));
    s->fpost = (double*)calloc(9 * n, sizeof(double));
    s->gpost = (double*)calloc(9 * n, sizeof(double));
    double** fields[] = {&s->rho, &s->phi, &s->ux, &s->uy, &s->phix, &s->dx, &s->dy, &s->lap};
    for (size_t k = 0; k < sizeof(fields) / sizeof(fields[0]); ++k)
        *fields[k] = (double*)calloc(n, sizeof(double));
    for (size_t r = 0; r < n; ++r) s->solid[r] = solid[r] ? 1 : 0;
    if (dphi) memcpy(s->dphi, dphi, n * sizeof(double));
    const int nx = p->nx, ny = p->ny;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const size_t r = (size_t)y * nx + x;
            if (s->solid[r]) continue;
            for (int k = 1; k < 9; ++k)
                if (s->solid[(size_t)wrap(y + EY[k], ny) * nx + wrap(x + EX[k], nx)])
                    s->boundary[r] = 1;
        }
    for (size_t r = 0; r < n; ++r) {
        const int fl = !s->solid[r];
        s->phi[r] = fl ? phi0[r] : 0.0;
        s->rho[r] = fl ? (rho0 ? rho0[r] : 1.0) : 0.0;
        s->ux[r] = fl && ux0 ? ux0[r] : 0.0;
        s->uy[r] = fl && uy0 ? uy0[r] : 0.0;
    }
    /* S_0: equilibria of the initial fields with their own velocity. */
    equilibria_field(s, 0, s->f, s->g);
    if (p->bounce == 1) {
        /* wall nodes: what the fluid equilibria send into them */
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                if (!is_wall(nx, ny, s->solid, x, y)) continue;
                const size_t w = (size_t)y * nx + x;
                for (int i = 1; i < 9; ++i) {
                    const size_t q = (size_t)wrap(y - EY[i], ny) * nx + wrap(x - EX[i], nx);
                    if (s->solid[q]) continue;
                    s->f[i * n + w] = s->f[i * n + q];
                    s->g[i * n + w] = s->g[i * n + q];
                }
            }
    }
    return s;
}

void orc_free(orc_state* s) {
    if (!s) return;
    free(s->solid);
    free(s->boundary);
    free(s->dphi);
    free(s->f);
    free(s->g);
    free(s->fpost);
    free(s->gpost);
    free(s->rho);
    free(s->phi);
    free(s->ux);
    free(s->uy);
    free(s->phix);
    free(s->dx);
    free(s->dy);
    free(s->lap);
    free(s);
}

void orc_step(orc_state* s, int64_t nsteps) {
    const orc_params* p = &s->p;
    const int nx = p->nx, ny = p->ny;
    const size_t n = s->n;
    for (int64_t t = 0; t < nsteps; ++t) {
        /* Step 1: moments, then the gradient terms the equilibria need. */
        orc_moments(nx, ny, s->solid, s->f, s->g, s->rho, s->phi, s->ux, s->uy);
        /* Step 2 (flag) and the equilibria, written straight into the post arrays. */
        equilibria_field(s, 1, s->fpost, s->gpost);
        /* Step 3: collision, node by node (fpost holds f^eq on entry). */
#pragma omp parallel for schedule(static)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const size_t r = (size_t)y * nx + x;
                if (s->solid[r]) continue;
                double f[9], g[9], feq[9], geq[9], fo[9], go[9];
                for (int i = 0; i < 9; ++i) {
                    f[i] = s->f[i * n + r];
                    g[i] = s->g[i * n + r];
                    feq[i] = s->fpost[i * n + r];
                    geq[i] = s->gpost[i * n + r];
                }
                orc_collide_node(p, s->phi[r], f, feq, g, geq, fo, go);
                for (int i = 0; i < 9; ++i) {
                    s->fpost[i * n + r] = fo[i];
                    s->gpost[i * n + r] = go[i];
                }
            }
        /* Step 4: streaming with bounce-back. */
        if (p->bounce == 1) {
            orc_reflect_walls(nx, ny, s->solid, s->f, s->fpost);
            orc_reflect_walls(nx, ny, s->solid, s->g, s->gpost);
            orc_stream_lattice_node(nx, ny, s->solid, s->fpost, s->f);
            orc_stream_lattice_node(nx, ny, s->solid, s->gpost, s->g);
        } else {
            orc_stream(nx, ny, s->solid, s->fpost, s->f);
            orc_stream(nx, ny, s->solid, s->gpost, s->g);
        }
        s->step += 1;
    }
}

int64_t orc_step_count(const orc_state* s) { return s->step; }

void orc_set_wall_dphi(orc_state* s, const double* dphi) {
    if (dphi)
        memcpy(s->dphi, dphi, s->n * sizeof(double));
    else
        memset(s->dphi, 0, s->n * sizeof(double));
}

void orc_fields(const orc_state* s, double* phi, double* rho, double* ux, double* uy) {
    orc_moments(s->p.nx, s->p.ny, s->solid, s->f, s->g, rho, phi, ux, uy);
}

void orc_get_populations(const orc_state* s, double* f, double* g) {
    if (f) memcpy(f, s->f, 9 * s->n * sizeof(double));
    if (g) memcpy(g, s->g, 9 * s->n * sizeof(double));
}

void orc_set_populations(orc_state* s, const double* f, const double* g) {
    if (f) memcpy(s->f, f, 9 * s->n * sizeof(double));
    if (g) memcpy(s->g, g, 9 * s->n * sizeof(double));
}

/* Neumaier compensated summation. */
typedef struct {
    double sum, comp;
} ksum;
static void ksum_add(ksum* k, double v) {
    const double t = k->sum + v;
    if (fabs(k->sum) >= fabs(v))
        k->comp += (k->sum - t) + v;
    else
        k->comp += (v - t) + k->sum;
    k->sum = t;
}

void orc_diagnostics(const orc_state* s, double out[5]) {
    const size_t n = s->n;
    double* rho = (double*)malloc(n * sizeof(double));
    double* phi = (double*)malloc(n * sizeof(double));
    double* ux = (double*)malloc(n * sizeof(double));
    double* uy = (double*)malloc(n * sizeof(double));
    orc_fields(s, phi, rho, ux, uy);
    ksum sr = {0, 0}, sp = {0, 0}, ke = {0, 0};
    double umax = 0.0, nf = 0.0;
    for (size_t r = 0; r < n; ++r) {
        if (s->solid[r]) continue;
        const double u2 = ux[r] * ux[r] + uy[r] * uy[r];
        ksum_add(&sr, rho[r]);
        ksum_add(&sp, phi[r]);
        ksum_add(&ke, 0.5 * rho[r] * u2);
        if (sqrt(u2) > umax || isnan(u2)) umax = sqrt(u2);
        nf += 1.0;
    }
    out[0] = sr.sum + sr.comp;
    out[1] = sp.sum + sp.comp;
    out[2] = ke.sum + ke.comp;
    out[3] = umax;
    out[4] = nf;
    free(rho);
    free(phi);
    free(ux);
    free(uy);
}

void orc_set_threads(int32_t n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int32_t orc_get_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
