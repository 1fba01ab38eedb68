/*
 * Stand-alone driver of the FP64 oracle for a build under AddressSanitizer and
 * UndefinedBehaviorSanitizer (TEST INFRASTRUCTURE, run only by the tests).
 *
 * The oracle is a shared library loaded by Python, where the sanitizers cannot
 * be preloaded; this program links lbm_oracle.c directly, so one instrumented
 * executable exercises every exported routine on one case and writes what it
 * computed, so the test can check the instrumented build against the ordinary
 * one bit for bit.
 *
 * usage: sanitize_driver <dir>
 *   <dir>/params.txt   nx ny A B kappa Gamma tau_alpha tau_beta tau_phi
 *                      collision zero_u_feq zero_u_geq tau_clamp tau_lut bounce steps
 *   <dir>/solid.u8     nx*ny bytes
 *   <dir>/dphi.f64, phi.f64, rho.f64, ux.f64, uy.f64   nx*ny doubles each
 * writes
 *   <dir>/out_f.f64, out_g.f64     S_steps, 9*nx*ny each
 *   <dir>/out_fields.f64           phi, rho, ux, uy of S_steps, 4*nx*ny
 *   <dir>/out_diag.f64             the five diagnostics
 *   <dir>/out_parts.f64            the individual steps applied to S_steps:
 *                                  moments (4 planes), ghosts, gradients (3),
 *                                  mid-link streaming (9), lattice-node streaming (9),
 *                                  wall reversal (9), then tau at 64 values of phi
 * exit status 0 on success, 2 on bad input, 3 if the oracle rejected the case.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lbm_oracle.h"

static void* read_file(const char* dir, const char* name, size_t bytes) {
    char path[4096];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE* fp = fopen(path, "rb");
    if (!fp) return NULL;
    void* buf = malloc(bytes ? bytes : 1);
    size_t got = buf ? fread(buf, 1, bytes, fp) : 0;
    fclose(fp);
    if (got != bytes) {
        free(buf);
        return NULL;
    }
    return buf;
}

static int write_file(const char* dir, const char* name, const void* data, size_t bytes) {
    char path[4096];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE* fp = fopen(path, "wb");
    if (!fp) return 0;
    size_t put = fwrite(data, 1, bytes, fp);
    return fclose(fp) == 0 && put == bytes;
}

int main(int argc, char** argv) {
    if (argc != 2) {
        fprintf(stderr, "usage: %s <dir>\n", argv[0]);
        return 2;
    }
    const char* dir = argv[1];
    char path[4096];
    snprintf(path, sizeof path, "%s/params.txt", dir);
    FILE* fp = fopen(path, "r");
    if (!fp) return 2;
    orc_params p;
    memset(&p, 0, sizeof p);
    long long steps = 0;
    int n = fscanf(fp, "%d %d %lf %lf %lf %lf %lf %lf %lf %d %d %d %d %d %d %lld", &p.nx, &p.ny,
                   &p.A, &p.B, &p.kappa, &p.Gamma, &p.tau_alpha, &p.tau_beta, &p.tau_phi,
                   &p.collision, &p.zero_u_feq, &p.zero_u_geq, &p.tau_clamp, &p.tau_lut,
                   &p.bounce, &steps);
    fclose(fp);
    if (n != 16 || p.nx < 1 || p.ny < 1 || steps < 0) return 2;

    const size_t N = (size_t)p.nx * (size_t)p.ny;
    uint8_t* solid = read_file(dir, "solid.u8", N);
    double* dphi = read_file(dir, "dphi.f64", N * sizeof(double));
    double* phi0 = read_file(dir, "phi.f64", N * sizeof(double));
    double* rho0 = read_file(dir, "rho.f64", N * sizeof(double));
    double* ux0 = read_file(dir, "ux.f64", N * sizeof(double));
    double* uy0 = read_file(dir, "uy.f64", N * sizeof(double));
    orc_state* s = NULL;
    if (solid && dphi && phi0 && rho0 && ux0 && uy0) {
        orc_set_threads(2);
        s = orc_create(&p, solid, dphi, phi0, rho0, ux0, uy0);
    }
    if (!s) {
        const int status = (solid && dphi && phi0 && rho0 && ux0 && uy0) ? 3 : 2;
        free(solid);
        free(dphi);
        free(phi0);
        free(rho0);
        free(ux0);
        free(uy0);
        return status;
    }
    /* half the steps, a wall-field update with the same values, the rest: the
       set-up routine is exercised without changing the result */
    orc_step(s, steps / 2);
    orc_set_wall_dphi(s, dphi);
    orc_step(s, steps - steps / 2);
    if (orc_step_count(s) != steps) return 4;

    double* f = malloc(9 * N * sizeof(double));
    double* g = malloc(9 * N * sizeof(double));
    double* fields = malloc(4 * N * sizeof(double));
    const size_t n_parts = 4 * N + N + 3 * N + 3 * 9 * N + 64;
    double* parts = malloc(n_parts * sizeof(double));
    double diag[5];
    if (!f || !g || !fields || !parts) return 2;
    orc_get_populations(s, f, g);
    orc_set_populations(s, f, g); /* a round trip that must change nothing */
    orc_get_populations(s, f, g);
    orc_fields(s, fields, fields + N, fields + 2 * N, fields + 3 * N);
    orc_diagnostics(s, diag);

    double* q = parts;
    orc_moments(p.nx, p.ny, solid, f, g, q, q + N, q + 2 * N, q + 3 * N);
    double* phi = q + N;
    q += 4 * N;
    orc_ghosts(p.nx, p.ny, solid, dphi, phi, q);
    double* phix = q;
    q += N;
    orc_gradients(p.nx, p.ny, solid, phix, q, q + N, q + 2 * N);
    q += 3 * N;
    orc_stream(p.nx, p.ny, solid, f, q);
    q += 9 * N;
    orc_stream_lattice_node(p.nx, p.ny, solid, f, q);
    q += 9 * N;
    memset(q, 0, 9 * N * sizeof(double));
    orc_reflect_walls(p.nx, p.ny, solid, f, q);
    q += 9 * N;
    for (int k = 0; k < 64; ++k) q[k] = orc_tau(&p, -1.6 + 3.2 * k / 63.0);

    int ok = write_file(dir, "out_f.f64", f, 9 * N * sizeof(double)) &&
             write_file(dir, "out_g.f64", g, 9 * N * sizeof(double)) &&
             write_file(dir, "out_fields.f64", fields, 4 * N * sizeof(double)) &&
             write_file(dir, "out_diag.f64", diag, sizeof diag) &&
             write_file(dir, "out_parts.f64", parts, n_parts * sizeof(double));
    orc_free(s);
    free(f);
    free(g);
    free(fields);
    free(parts);
    free(solid);
    free(dphi);
    free(phi0);
    free(rho0);
    free(ux0);
    free(uy0);
    return ok ? 0 : 2;
}
