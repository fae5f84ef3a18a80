/*
 * adref -- plain FP64 CPU oracle for suspensions of active spring dumbbells.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library. The GPU library never
 * links, includes or calls it, and the two share no code.
 *
 * What it computes (Putz, Dunkel, Yeomans, "CUDA simulations of active
 * dumbbell suspensions"):
 *   - Deterministic overdamped dynamics, Sec. II, Eq. (e:langevin) at zero
 *     temperature:  dX_i/dt = sum_j H_ij F_j.
 *   - Mobility H, Sec. II, Eq. (e:Mazur): self term I/(6 pi eta a) and the
 *     Oseen pair tensor (I + rr/r^2)/(8 pi eta r), r = X_i - X_j (first line of
 *     Eq. e:Mazur_offdiagonal; the Oseen approximation stated after it).
 *     Optionally the Rotne-Prager-Yamakawa-Mazur correction of the second
 *     line, 2a^2/(24 pi eta r^3) (I - 3 rr/r^2).
 *   - Spring forces, Sec. II, Eq. (e:swimmer_potential): U = k/2 (d - L(t))^2
 *     per dumbbell with L(t) = ell + lam sin(omega t + phi), F = -grad U.
 *     Dumbbell s owns spheres 2s and 2s+1 (0-based); the force on sphere 2s+1
 *     is -k (d - L) n/d with n = X_{2s+1} - X_{2s}, and sphere 2s gets its
 *     negative.
 *   - Optional steric repulsion (not in the paper): for r < rc each sphere i
 *     gets steric_k (rc - r) (X_i - X_j)/r from each sphere j.
 *   - Time stepping: classical RK4 (default) or the paper's Heun
 *     predictor-corrector (Sec. V), x~ = x + dt u(x,t),
 *     x' = x + dt/2 (u(x,t) + u(x~,t+dt)).
 *   - Optional Brownian noise with Heun: the additive form with a constant
 *     matrix C the paper recommends for dilute suspensions (Sec. V). With H
 *     replaced by its diagonal, 2H = C C^T (Eq. e:cholesky) gives
 *     C = sqrt(2/(6 pi eta a)) I, so both Heun stages add
 *     sqrt(2 kT dt/(6 pi eta a)) xi with the same standard normal xi.
 *     xi comes from the counter-based generator Philox4x32-10 (Salmon,
 *     Moraes, Dror, Shaw, SC'11), key = seed, counter = (sphere, step), and
 *     the Box-Muller transform.
 *
 * Readings where the paper leaves freedom (each is fixed here on purpose):
 *   - sin(omega t + phi) is evaluated by the addition theorem,
 *     sin(omega t) cos(phi) + cos(omega t) sin(phi), with libm sin/cos.
 *   - Step n starts at t_n = t0 + n*dt (never accumulated); RK4 stage times
 *     are t_n, t_n + dt/2, t_n + dt/2, t_n + dt.
 *   - Sums over j run in ascending j over all j != i, partner included; a
 *     pair at zero distance contributes nothing and is counted as an error.
 *   - Built without fast-math and without FMA contraction.
 *
 * Mobility is a plain double loop, parallel over i only, so the result does
 * not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ADREF_OK 0
#define ADREF_EINVAL (-1)
#define ADREF_ENOMEM (-2)
#define ADREF_ENONFINITE (-5)

typedef struct adref_params {
    double a, eta, k, ell, lam, T, dt;
    double steric_k, steric_r;
    int32_t integrator; /* 0 = RK4, 1 = Heun */
    int32_t tensor;     /* 0 = Oseen, 1 = Oseen + RPY-Mazur correction */
    double kT;          /* thermal energy k_B T (0: deterministic; Heun only) */
    uint64_t seed;      /* key of the noise generator */
} adref_params;

static const double PI = 3.14159265358979323846;

void adref_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int adref_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Philox4x32-10: ten rounds of two 32x32->64 multiplications with the
 * published multipliers, the key bumped by the Weyl constants between
 * rounds. */
static void philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void adref_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    philox4x32_10(ctr, key, out);
}

/* Three standard normals for sphere i at step n: Box-Muller on the four
 * uniforms (x + 1/2) 2^-32 of one Philox block. */
static void gauss3(uint64_t seed, int64_t i, int64_t n, double z[3]) {
    uint32_t ctr[4] = {(uint32_t)i, (uint32_t)n, (uint32_t)((uint64_t)n >> 32), 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    philox4x32_10(ctr, key, x);
    double u[4];
    for (int q = 0; q < 4; ++q) u[q] = ((double)x[q] + 0.5) / 4294967296.0;
    double r0 = sqrt(-2.0 * log(u[0])), r1 = sqrt(-2.0 * log(u[2]));
    z[0] = r0 * cos((2.0 * PI) * u[1]);
    z[1] = r0 * sin((2.0 * PI) * u[1]);
    z[2] = r1 * cos((2.0 * PI) * u[3]);
}

void adref_gauss3(uint64_t seed, int64_t i, int64_t n, double z[3]) { gauss3(seed, i, n, z); }

/* Rest length L(t) of dumbbell s (Eq. e:swimmer_potential). */
static double rest_length(const adref_params* p, double t, double phi) {
    double omega = 2.0 * PI / p->T;
    double wt = omega * t;
    double st = sin(wt), ct = cos(wt);
    double sphi = sin(phi), cphi = cos(phi);
    return p->ell + p->lam * (st * cphi + ct * sphi);
}

double adref_rest_length(const adref_params* p, double t, double phi) {
    return rest_length(p, t, phi);
}

/* F = -grad U for one system of N = 2S spheres; steric pairs added after. */
int adref_forces(const adref_params* p, int64_t N, const double* X, const double* phi,
                 double t, double* F) {
    if (!p || !X || !phi || !F || N < 0 || (N & 1)) return ADREF_EINVAL;
    int64_t S = N / 2;
    for (int64_t s = 0; s < S; ++s) {
        const double* x0 = X + 3 * (2 * s);
        const double* x1 = X + 3 * (2 * s + 1);
        double nx = x1[0] - x0[0], ny = x1[1] - x0[1], nz = x1[2] - x0[2];
        double d = sqrt((nx * nx + ny * ny) + nz * nz);
        double L = rest_length(p, t, phi[s]);
        double c = -p->k * (d - L) / d;
        double fx = c * nx, fy = c * ny, fz = c * nz;
        F[3 * (2 * s + 1) + 0] = fx;
        F[3 * (2 * s + 1) + 1] = fy;
        F[3 * (2 * s + 1) + 2] = fz;
        F[3 * (2 * s) + 0] = -fx;
        F[3 * (2 * s) + 1] = -fy;
        F[3 * (2 * s) + 2] = -fz;
    }
    int bad = 0;
    if (p->steric_k != 0.0) {
        double rc = p->steric_r, rc2 = rc * rc;
        /* Accumulate into a copy so every sphere sees the spring-only forces
         * plus its own ascending-j steric sum. */
        #pragma omp parallel for schedule(static) reduction(+:bad)
        for (int64_t i = 0; i < N; ++i) {
            double ax = 0.0, ay = 0.0, az = 0.0;
            int any = 0;
            for (int64_t j = 0; j < N; ++j) {
                if (j == i) continue;
                double rx = X[3 * i + 0] - X[3 * j + 0];
                double ry = X[3 * i + 1] - X[3 * j + 1];
                double rz = X[3 * i + 2] - X[3 * j + 2];
                double r2 = (rx * rx + ry * ry) + rz * rz;
                if (r2 >= rc2) continue;
                if (r2 == 0.0) { bad += 1; continue; }
                double r = sqrt(r2);
                double c = p->steric_k * (rc - r) / r;
                ax = ax + c * rx;
                ay = ay + c * ry;
                az = az + c * rz;
                any = 1;
            }
            if (any) {
                F[3 * i + 0] = F[3 * i + 0] + ax;
                F[3 * i + 1] = F[3 * i + 1] + ay;
                F[3 * i + 2] = F[3 * i + 2] + az;
            }
        }
    }
    return bad ? ADREF_ENONFINITE : ADREF_OK;
}

/* Spring energy U = sum_s k/2 (d_s - L_s(t))^2. */
double adref_energy(const adref_params* p, int64_t N, const double* X, const double* phi, double t) {
    double U = 0.0;
    for (int64_t s = 0; s < N / 2; ++s) {
        const double* x0 = X + 3 * (2 * s);
        const double* x1 = X + 3 * (2 * s + 1);
        double nx = x1[0] - x0[0], ny = x1[1] - x0[1], nz = x1[2] - x0[2];
        double d = sqrt((nx * nx + ny * ny) + nz * nz);
        double e = d - rest_length(p, t, phi[s]);
        U = U + 0.5 * p->k * e * e;
    }
    return U;
}

/* u_i = F_i/(6 pi eta a) + 1/(8 pi eta) sum_{j != i} [F_j/r + r (r.F_j)/r^3]
 * (+ RPY correction when tensor == 1). Returns the number of coincident
 * pairs met (they contribute zero). */
static int64_t mobility_row(const adref_params* p, int64_t N, const double* X, const double* F,
                            int64_t i, double* ui) {
    double cs = 1.0 / (6.0 * PI * p->eta * p->a);
    double co = 1.0 / (8.0 * PI * p->eta);
    double xi = X[3 * i + 0], yi = X[3 * i + 1], zi = X[3 * i + 2];
    double ax = 0.0, ay = 0.0, az = 0.0;
    double bx = 0.0, by = 0.0, bz = 0.0;
    int64_t bad = 0;
    for (int64_t j = 0; j < N; ++j) {
        if (j == i) continue;
        double rx = xi - X[3 * j + 0];
        double ry = yi - X[3 * j + 1];
        double rz = zi - X[3 * j + 2];
        double r2 = (rx * rx + ry * ry) + rz * rz;
        if (r2 == 0.0) { bad += 1; continue; }
        double Fx = F[3 * j + 0], Fy = F[3 * j + 1], Fz = F[3 * j + 2];
        double ir = 1.0 / sqrt(r2);
        double fr = (rx * Fx + ry * Fy) + rz * Fz;
        double t = fr / r2;
        ax = ax + ir * (Fx + t * rx);
        ay = ay + ir * (Fy + t * ry);
        az = az + ir * (Fz + t * rz);
        if (p->tensor == 1) {
            /* (I - 3 rr/r^2) F / r^3 */
            double ir3 = ir / r2;
            double t3 = 3.0 * t;
            bx = bx + ir3 * (Fx - t3 * rx);
            by = by + ir3 * (Fy - t3 * ry);
            bz = bz + ir3 * (Fz - t3 * rz);
        }
    }
    ui[0] = cs * F[3 * i + 0] + co * ax;
    ui[1] = cs * F[3 * i + 1] + co * ay;
    ui[2] = cs * F[3 * i + 2] + co * az;
    if (p->tensor == 1) {
        double cr = 2.0 * p->a * p->a / (24.0 * PI * p->eta);
        ui[0] = ui[0] + cr * bx;
        ui[1] = ui[1] + cr * by;
        ui[2] = ui[2] + cr * bz;
    }
    return bad;
}

int adref_mobility(const adref_params* p, int64_t N, const double* X, const double* F, double* u) {
    if (!p || !X || !F || !u || N < 0) return ADREF_EINVAL;
    int64_t bad = 0;
    #pragma omp parallel for schedule(static) reduction(+:bad)
    for (int64_t i = 0; i < N; ++i) bad += mobility_row(p, N, X, F, i, u + 3 * i);
    return bad ? ADREF_ENONFINITE : ADREF_OK;
}

/* The names of the library's calls: adref_mobility_apply is adref_mobility
 * (u = M(X) F for caller forces), adref_step is adref_run without records
 * (the oracle keeps no state: X is advanced in place). */
int adref_mobility_apply(const adref_params* p, int64_t N, const double* X, const double* F, double* u) {
    return adref_mobility(p, N, X, F, u);
}

int adref_run(const adref_params* p, int32_t nsys, const int64_t* off, double* X, const double* phi,
              double t0, int64_t step0, int64_t nsteps, int64_t record_every,
              double* centres_out, double* com_out);

int adref_step(const adref_params* p, int32_t nsys, const int64_t* off, double* X, const double* phi,
               double t0, int64_t step0, int64_t nsteps) {
    return adref_run(p, nsys, off, X, phi, t0, step0, nsteps, 0, NULL, NULL);
}

/* The same sum for a subset of target spheres: u_rows[r] = u_{rows[r]}. */
int adref_mobility_rows(const adref_params* p, int64_t N, const double* X, const double* F,
                        int64_t nrows, const int64_t* rows, double* u_rows) {
    if (!p || !X || !F || !rows || !u_rows || N < 0 || nrows < 0) return ADREF_EINVAL;
    for (int64_t r = 0; r < nrows; ++r)
        if (rows[r] < 0 || rows[r] >= N) return ADREF_EINVAL;
    int64_t bad = 0;
    #pragma omp parallel for schedule(static) reduction(+:bad)
    for (int64_t r = 0; r < nrows; ++r) bad += mobility_row(p, N, X, F, rows[r], u_rows + 3 * r);
    return bad ? ADREF_ENONFINITE : ADREF_OK;
}

/* Brute force: assemble the dense 3N x 3N tensor H, then u = H F. */
int adref_mobility_dense(const adref_params* p, int64_t N, const double* X, const double* F, double* u) {
    if (!p || !X || !F || !u || N < 0 || N > 4096) return ADREF_EINVAL;
    int64_t M = 3 * N;
    double* H = (double*)calloc((size_t)(M * M), sizeof(double));
    if (!H) return ADREF_ENOMEM;
    double cs = 1.0 / (6.0 * PI * p->eta * p->a);
    double co = 1.0 / (8.0 * PI * p->eta);
    double cr = 2.0 * p->a * p->a / (24.0 * PI * p->eta);
    int bad = 0;
    for (int64_t i = 0; i < N; ++i) {
        for (int64_t j = 0; j < N; ++j) {
            double* blk = H + (3 * i) * M + 3 * j;
            if (i == j) {
                for (int a = 0; a < 3; ++a) blk[a * M + a] = cs;
                continue;
            }
            double r[3];
            for (int a = 0; a < 3; ++a) r[a] = X[3 * i + a] - X[3 * j + a];
            double rr = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
            if (rr == 0.0) { bad = 1; continue; }
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    double delta = (a == b) ? 1.0 : 0.0;
                    double h = co / rr * (delta + r[a] * r[b] / (rr * rr));
                    if (p->tensor == 1) h += cr / (rr * rr * rr) * (delta - 3.0 * r[a] * r[b] / (rr * rr));
                    blk[a * M + b] = h;
                }
        }
    }
    for (int64_t r = 0; r < M; ++r) {
        double s = 0.0;
        for (int64_t c = 0; c < M; ++c) s += H[r * M + c] * F[c];
        u[r] = s;
    }
    free(H);
    return bad ? ADREF_ENONFINITE : ADREF_OK;
}

/* Velocity field u(X, t) = H(X) F(X, t) for one system. */
static int velocity(const adref_params* p, int64_t N, const double* X, const double* phi, double t,
                    double* F, double* u, int threaded) {
    int st = adref_forces(p, N, X, phi, t, F);
    int64_t bad = 0;
    if (threaded) {
        #pragma omp parallel for schedule(static) reduction(+:bad)
        for (int64_t i = 0; i < N; ++i) bad += mobility_row(p, N, X, F, i, u + 3 * i);
    } else {
        for (int64_t i = 0; i < N; ++i) bad += mobility_row(p, N, X, F, i, u + 3 * i);
    }
    return (st != ADREF_OK || bad) ? ADREF_ENONFINITE : ADREF_OK;
}

static int all_finite(const double* v, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

/* Advance one system by nsteps from step index step0; records every
 * record_every steps (centres [S][3] and COM [3] per record, strided). */
static int advance_system(const adref_params* p, int64_t N, double* X, const double* phi, double t0,
                          int64_t step0, int64_t nsteps, int64_t record_every,
                          double* centres, int64_t centre_stride, double* com, int64_t com_stride,
                          int threaded, int64_t ioff) {
    int64_t M = 3 * N;
    double* buf = (double*)malloc(sizeof(double) * (size_t)(M * 7 + 1));
    if (!buf) return ADREF_ENOMEM;
    double *F = buf, *k1 = buf + M, *k2 = buf + 2 * M, *k3 = buf + 3 * M, *k4 = buf + 4 * M;
    double* Y = buf + 5 * M;
    double* xi = buf + 6 * M;
    const double g = sqrt(2.0 * p->kT * (1.0 / (6.0 * PI * p->eta * p->a)) * p->dt);
    int status = ADREF_OK;
    double dt = p->dt;
    int64_t rec = 0;
    for (int64_t n = 0; n < nsteps; ++n) {
        int64_t step = step0 + n;
        double tn = t0 + (double)step * dt;
        int st = 0;
        if (p->integrator == 1) {
            /* Heun predictor-corrector, with the same noise in both stages */
            if (p->kT > 0.0)
                for (int64_t i = 0; i < N; ++i) gauss3(p->seed, ioff + i, step, xi + 3 * i);
            st |= velocity(p, N, X, phi, tn, F, k1, threaded);
            if (p->kT > 0.0)
                for (int64_t c = 0; c < M; ++c) Y[c] = (X[c] + dt * k1[c]) + g * xi[c];
            else
                for (int64_t c = 0; c < M; ++c) Y[c] = X[c] + dt * k1[c];
            st |= velocity(p, N, Y, phi, tn + dt, F, k2, threaded);
            if (p->kT > 0.0)
                for (int64_t c = 0; c < M; ++c) X[c] = (X[c] + (0.5 * dt) * (k1[c] + k2[c])) + g * xi[c];
            else
                for (int64_t c = 0; c < M; ++c) X[c] = X[c] + (0.5 * dt) * (k1[c] + k2[c]);
        } else {
            double th = tn + 0.5 * dt, te = tn + dt;
            st |= velocity(p, N, X, phi, tn, F, k1, threaded);
            for (int64_t c = 0; c < M; ++c) Y[c] = X[c] + (0.5 * dt) * k1[c];
            st |= velocity(p, N, Y, phi, th, F, k2, threaded);
            for (int64_t c = 0; c < M; ++c) Y[c] = X[c] + (0.5 * dt) * k2[c];
            st |= velocity(p, N, Y, phi, th, F, k3, threaded);
            for (int64_t c = 0; c < M; ++c) Y[c] = X[c] + dt * k3[c];
            st |= velocity(p, N, Y, phi, te, F, k4, threaded);
            for (int64_t c = 0; c < M; ++c)
                X[c] = X[c] + (dt / 6.0) * (((k1[c] + 2.0 * k2[c]) + 2.0 * k3[c]) + k4[c]);
        }
        if (st != ADREF_OK) status = ADREF_ENONFINITE;
        if (record_every > 0 && (n + 1) % record_every == 0) {
            if (!all_finite(X, M)) status = ADREF_ENONFINITE;
            if (centres) {
                double* c = centres + rec * centre_stride;
                for (int64_t s = 0; s < N / 2; ++s)
                    for (int a = 0; a < 3; ++a)
                        c[3 * s + a] = 0.5 * (X[3 * (2 * s) + a] + X[3 * (2 * s + 1) + a]);
            }
            if (com) {
                double* m = com + rec * com_stride;
                for (int a = 0; a < 3; ++a) {
                    double sum = 0.0;
                    for (int64_t i = 0; i < N; ++i) sum = sum + X[3 * i + a];
                    m[a] = sum / (double)N;
                }
            }
            ++rec;
        }
    }
    if (!all_finite(X, M)) status = ADREF_ENONFINITE;
    free(buf);
    return status;
}

/* Advance nsys independent systems (sphere offsets off[nsys+1]) in place.
 * centres_out: [nrec][S_total][3]; com_out: [nrec][nsys][3], nrec =
 * nsteps / record_every; either may be NULL. */
int adref_run(const adref_params* p, int32_t nsys, const int64_t* off, double* X, const double* phi,
              double t0, int64_t step0, int64_t nsteps, int64_t record_every,
              double* centres_out, double* com_out) {
    if (!p || !off || !X || !phi || nsys <= 0 || nsteps < 0 || record_every < 0) return ADREF_EINVAL;
    if (p->kT < 0.0 || (p->kT > 0.0 && p->integrator != 1)) return ADREF_EINVAL;
    for (int32_t b = 0; b < nsys; ++b)
        if (off[b + 1] < off[b] || ((off[b + 1] - off[b]) & 1) || (off[b] & 1)) return ADREF_EINVAL;
    int64_t S_total = off[nsys] / 2;
    int status = ADREF_OK;
    if (nsys == 1) {
        return advance_system(p, off[1] - off[0], X + 3 * off[0], phi + off[0] / 2, t0, step0, nsteps,
                              record_every, centres_out, 3 * S_total, com_out, 3, 1, off[0]);
    }
    #pragma omp parallel for schedule(dynamic, 1)
    for (int32_t b = 0; b < nsys; ++b) {
        int64_t N = off[b + 1] - off[b];
        int st = advance_system(p, N, X + 3 * off[b], phi + off[b] / 2, t0, step0, nsteps, record_every,
                                centres_out ? centres_out + 3 * (off[b] / 2) : NULL, 3 * S_total,
                                com_out ? com_out + 3 * b : NULL, 3 * (int64_t)nsys, 0, off[b]);
        if (st != ADREF_OK) {
            #pragma omp critical
            status = st;
        }
    }
    return status;
}

/* ------------------------------------------------------------------------
 * Stroke-averaged far-field equations (Sec. III, Eqs. e:eom, J, K and the
 * projections s, r, q): for dumbbells with centres R, unit axes N and phases
 * phi,
 *   dR_s/dt = sum_{r != s} J^{sr},   dN_s/dt = -(I - N_s N_s) sum_{r != s} K^{sr},
 *   J^{sr} = a w sin(phi_s - phi_r) (9/64) (lam/ell)^2 (ell/D)^4
 *            { N_s (2s + 4qr - 10 s r^2)
 *              + Dhat (1 + 2q^2 - 5s^2 - 5r^2 - 20 q s r + 35 s^2 r^2) },
 *   K^{sr} = w sin(phi_s - phi_r) (15/64) (a/ell) (lam/ell)^2 (ell/D)^5 Dhat
 *            (3s + 6rq + 6 s q^2 - 7 s^3 - 21 s r^2 - 42 q s^2 r + 63 s^3 r^2),
 *   D = R_s - R_r, s = Dhat.N_s, r = Dhat.N_r, q = N_s.N_r, w = 2 pi/T.
 * Sums in ascending r. The equations are autonomous.
 * ------------------------------------------------------------------------ */
int adref_sa_rhs(const adref_params* p, int64_t S, const double* R, const double* N, const double* phi,
                 double* dR, double* dN) {
    if (!p || !R || !N || !phi || !dR || !dN || S < 0) return ADREF_EINVAL;
    double w = 2.0 * PI / p->T;
    double lr = p->lam / p->ell;
    double cj = p->a * w * (9.0 / 64.0) * lr * lr;
    double ck = w * (15.0 / 64.0) * (p->a / p->ell) * lr * lr;
    int bad = 0;
    #pragma omp parallel for schedule(static) reduction(+:bad)
    for (int64_t i = 0; i < S; ++i) {
        const double* ni = N + 3 * i;
        double jx = 0.0, jy = 0.0, jz = 0.0, kx = 0.0, ky = 0.0, kz = 0.0;
        for (int64_t j = 0; j < S; ++j) {
            if (j == i) continue;
            const double* nj = N + 3 * j;
            double Dx = R[3 * i + 0] - R[3 * j + 0];
            double Dy = R[3 * i + 1] - R[3 * j + 1];
            double Dz = R[3 * i + 2] - R[3 * j + 2];
            double D = sqrt((Dx * Dx + Dy * Dy) + Dz * Dz);
            if (D == 0.0) { bad = 1; continue; }
            double ux = Dx / D, uy = Dy / D, uz = Dz / D;
            double s = (ux * ni[0] + uy * ni[1]) + uz * ni[2];
            double r = (ux * nj[0] + uy * nj[1]) + uz * nj[2];
            double q = (ni[0] * nj[0] + ni[1] * nj[1]) + ni[2] * nj[2];
            double sn = sin(phi[i] - phi[j]);
            double x = p->ell / D;
            double x4 = (x * x) * (x * x);
            double aN = 2.0 * s + 4.0 * q * r - 10.0 * s * r * r;
            double aD = 1.0 + 2.0 * q * q - 5.0 * s * s - 5.0 * r * r - 20.0 * q * s * r + 35.0 * s * s * r * r;
            double fj = cj * sn * x4;
            jx = jx + fj * (ni[0] * aN + ux * aD);
            jy = jy + fj * (ni[1] * aN + uy * aD);
            jz = jz + fj * (ni[2] * aN + uz * aD);
            double bK = 3.0 * s + 6.0 * r * q + 6.0 * s * q * q - 7.0 * s * s * s - 21.0 * s * r * r
                        - 42.0 * q * s * s * r + 63.0 * s * s * s * r * r;
            double fk = ck * sn * (x4 * x) * bK;
            kx = kx + fk * ux;
            ky = ky + fk * uy;
            kz = kz + fk * uz;
        }
        dR[3 * i + 0] = jx;
        dR[3 * i + 1] = jy;
        dR[3 * i + 2] = jz;
        double nk = (ni[0] * kx + ni[1] * ky) + ni[2] * kz;
        dN[3 * i + 0] = -(kx - ni[0] * nk);
        dN[3 * i + 1] = -(ky - ni[1] * nk);
        dN[3 * i + 2] = -(kz - ni[2] * nk);
    }
    return bad ? ADREF_ENONFINITE : ADREF_OK;
}

/* RK4 on (R, N) with time step dt; after each step every axis is scaled back
 * to unit length (the exact flow keeps |N| = 1, RK4 only to O(dt^5)). */
int adref_sa_run(const adref_params* p, int64_t S, double* R, double* N, const double* phi, double dt,
                 int64_t nsteps) {
    if (!p || !R || !N || !phi || S < 0 || nsteps < 0 || !(dt > 0)) return ADREF_EINVAL;
    int64_t M = 3 * S;
    double* buf = (double*)malloc(sizeof(double) * (size_t)(M * 12 + 1));
    if (!buf) return ADREF_ENOMEM;
    double *kR[4], *kN[4];
    for (int s = 0; s < 4; ++s) {
        kR[s] = buf + (2 * s) * M;
        kN[s] = buf + (2 * s + 1) * M;
    }
    double *YR = buf + 8 * M, *YN = buf + 9 * M;
    int status = ADREF_OK;
    for (int64_t n = 0; n < nsteps; ++n) {
        status |= adref_sa_rhs(p, S, R, N, phi, kR[0], kN[0]);
        for (int64_t c = 0; c < M; ++c) { YR[c] = R[c] + (0.5 * dt) * kR[0][c]; YN[c] = N[c] + (0.5 * dt) * kN[0][c]; }
        status |= adref_sa_rhs(p, S, YR, YN, phi, kR[1], kN[1]);
        for (int64_t c = 0; c < M; ++c) { YR[c] = R[c] + (0.5 * dt) * kR[1][c]; YN[c] = N[c] + (0.5 * dt) * kN[1][c]; }
        status |= adref_sa_rhs(p, S, YR, YN, phi, kR[2], kN[2]);
        for (int64_t c = 0; c < M; ++c) { YR[c] = R[c] + dt * kR[2][c]; YN[c] = N[c] + dt * kN[2][c]; }
        status |= adref_sa_rhs(p, S, YR, YN, phi, kR[3], kN[3]);
        for (int64_t c = 0; c < M; ++c) {
            R[c] = R[c] + (dt / 6.0) * (((kR[0][c] + 2.0 * kR[1][c]) + 2.0 * kR[2][c]) + kR[3][c]);
            N[c] = N[c] + (dt / 6.0) * (((kN[0][c] + 2.0 * kN[1][c]) + 2.0 * kN[2][c]) + kN[3][c]);
        }
        for (int64_t i = 0; i < S; ++i) {
            double* v = N + 3 * i;
            double nn = sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
            v[0] = v[0] / nn;
            v[1] = v[1] / nn;
            v[2] = v[2] / nn;
        }
    }
    free(buf);
    return status ? ADREF_ENONFINITE : ADREF_OK;
}
