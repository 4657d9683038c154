/*
 * Plain FP64 CPU oracle for the lattice Boltzmann scheme for quasi-static
 * linear elasticity in 2D on periodic lattices (Boolakee, Geier, De Lorenzis,
 * "A new lattice Boltzmann scheme for linear elastic solids: periodic
 * problems", arXiv 2208.14870).
 *
 * THIS FILE IS TEST INFRASTRUCTURE.  It is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or constant with the GPU library.
 *
 * What it computes (lattice units: dx = dt = 1):
 *   - Velocity set: D2Q9 without the rest population (D2Q8), in the one-index
 *     order of the population table of Sec. 5 (Table "velocities"):
 *       1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1) 6:(-1,1) 7:(-1,-1) 8:(1,-1).
 *     The rest population only feeds m00, which no equilibrium or relaxed
 *     moment reads (Sec. 3.3.2, remarks after the relaxation-time matching),
 *     so it is not carried.
 *   - One time step = Algorithm 1: for every node compute the raw countable
 *     moments (Eq. moments) and the spherical/deviatoric pair (Eq.
 *     replace_raw); apply half of the forcing to the first-order moments
 *     (Eqs. coll10/coll01); build the equilibria of Table "scheme" from the
 *     bared first-order moments; relax every moment of the collision set
 *     (Eq. collision); apply the second half of the forcing (Eqs.
 *     coll10post/coll01post); solve Eq. moments_post for the post-collision
 *     populations; then stream (Eq. streaming) with periodic wrap (Sec. 6.1).
 *   - Observables: displacement = bared first-order moments (Table
 *     "solution", Sec. 7.1); stress from the bared second-order moments
 *     (Eq. compute_bared and Table "solution", in lattice units without the
 *     1/eps factor); the steady-state residual.
 *
 * Layout of a population field: f[q][y][x], q = 0..7 for populations 1..8,
 * x fastest, plane size nx*ny.  Every routine is plain loops; the collide and
 * stream passes are separate, as in Algorithm 1.  The only parallelism is an
 * OpenMP loop over rows, which does not change any result.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Microscopic velocities c_q = (CX[q], CY[q]) in the one-index order. */
static const int CX[8] = {1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[8] = {0, 1, 0, -1, 1, 1, -1, -1};

/* Index of each moment in the collision vector, in the one-index order of
 * the moment table of Sec. 5 (Table "moments"): 10, 01, 11, s, d, 12, 21, 22. */
enum { M10 = 0, M01 = 1, M11 = 2, MS = 3, MD = 4, M12 = 5, M21 = 6, M22 = 7 };

static double ipow(int base, int e) {
    double r = 1.0;
    for (int k = 0; k < e; ++k) r *= (double)base;
    return r;
}

/* Raw countable moment m_ab = sum_q i^a j^b f_q  (Eq. moments). */
static double raw_moment(const double f[8], int a, int b) {
    double m = 0.0;
    for (int q = 0; q < 8; ++q) m += ipow(CX[q], a) * ipow(CY[q], b) * f[q];
    return m;
}

/* Moments of the collision set in the one-index order, using Eq. replace_raw
 * for the spherical and deviatoric moments. */
static void moments(const double f[8], double m[8]) {
    double m20 = raw_moment(f, 2, 0);
    double m02 = raw_moment(f, 0, 2);
    m[M10] = raw_moment(f, 1, 0);
    m[M01] = raw_moment(f, 0, 1);
    m[M11] = raw_moment(f, 1, 1);
    m[MS] = m20 + m02;
    m[MD] = m20 - m02;
    m[M12] = raw_moment(f, 1, 2);
    m[M21] = raw_moment(f, 2, 1);
    m[M22] = raw_moment(f, 2, 2);
}

/* The 8x8 transform m = M f, assembled by applying moments() to unit vectors,
 * and its inverse by Gauss-Jordan elimination with partial pivoting.  The
 * inverse is what "solve Eq. moments_post for f*" amounts to. */
static double g_M[8][8], g_Minv[8][8];
static int g_ready = 0;

static void build_transform(void) {
    if (g_ready) return;
    for (int j = 0; j < 8; ++j) {
        double e[8] = {0}, m[8];
        e[j] = 1.0;
        moments(e, m);
        for (int i = 0; i < 8; ++i) g_M[i][j] = m[i];
    }
    double a[8][16];
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 16; ++j)
            a[i][j] = (j < 8) ? g_M[i][j] : (j - 8 == i ? 1.0 : 0.0);
    for (int c = 0; c < 8; ++c) {
        int p = c;
        for (int r = c + 1; r < 8; ++r)
            if (fabs(a[r][c]) > fabs(a[p][c])) p = r;
        if (p != c)
            for (int j = 0; j < 16; ++j) {
                double t = a[c][j]; a[c][j] = a[p][j]; a[p][j] = t;
            }
        double piv = a[c][c];
        for (int j = 0; j < 16; ++j) a[c][j] /= piv;
        for (int r = 0; r < 8; ++r) {
            if (r == c) continue;
            double fac = a[r][c];
            if (fac != 0.0)
                for (int j = 0; j < 16; ++j) a[r][j] -= fac * a[c][j];
        }
    }
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j) g_Minv[i][j] = a[i][j + 8];
    g_ready = 1;
}

/* ---------------------------------------------------------------------- */
/* Parameters                                                              */
/* ---------------------------------------------------------------------- */

/* Relaxation rates from the Lame parameters (lattice units) per Table
 * "scheme": tau_11 = mu/theta, tau_s = 2K/(1+theta), tau_d = 2mu/(1-theta),
 * K = lambda + mu, and omega = 1/(tau + 1/2) (Eq. relaxation_rate).
 * out = {omega_11, omega_s, omega_d}.  Returns 0, or -1 if mu <= 0,
 * K <= 0 or theta outside (0,1). */
int oracle_rates(double lame_lambda, double lame_mu, double theta, double out[3]) {
    double K = lame_lambda + lame_mu;
    if (!(lame_mu > 0.0) || !(K > 0.0) || !(theta > 0.0) || !(theta < 1.0)) return -1;
    double tau11 = lame_mu / theta;
    double taus = 2.0 * K / (1.0 + theta);
    double taud = 2.0 * lame_mu / (1.0 - theta);
    out[0] = 1.0 / (tau11 + 0.5);
    out[1] = 1.0 / (taus + 0.5);
    out[2] = 1.0 / (taud + 0.5);
    return 0;
}

/* The full relaxation-rate vector in the moment one-index order, with the
 * standard choice omega_12 = omega_21 = omega_22 = 1 of Sec. 3.3.2 unless
 * given.  omega_10 = omega_01 = 0 (first-order moments are not relaxed, only
 * forced).  out[8]. */
void oracle_omega_vector(double w11, double ws, double wd, double w12, double w21,
                         double w22, double out[8]) {
    out[M10] = 0.0;
    out[M01] = 0.0;
    out[M11] = w11;
    out[MS] = ws;
    out[MD] = wd;
    out[M12] = w12;
    out[M21] = w21;
    out[M22] = w22;
}

/* The moment transform as assembled above (row-major 8x8), for checking
 * against the matrix printed in Sec. 5. */
void oracle_moment_matrix(double out[64]) {
    build_transform();
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j) out[8 * i + j] = g_M[i][j];
}

/* ---------------------------------------------------------------------- */
/* Collision of one node (Algorithm 1, collision block)                   */
/* ---------------------------------------------------------------------- */

/* f[8] pre-collision populations, (gx, gy) forcing of this node, omega[8] in
 * moment order, theta the third-order equilibrium constant.  Writes the
 * post-collision populations fstar[8] and, if non-NULL, the bared
 * first-order moments (the displacement) u[2]. */
void oracle_collide_node(const double f[8], double gx, double gy, const double omega[8],
                         double theta, double fstar[8], double u[2]) {
    build_transform();
    double m[8], meq[8], mstar[8];
    moments(f, m);                                   /* compute moments        */
    double mb10 = m[M10] + 0.5 * gx;                 /* half forcing (coll10)  */
    double mb01 = m[M01] + 0.5 * gy;                 /* half forcing (coll01)  */
    if (u) { u[0] = mb10; u[1] = mb01; }             /* solution fields        */
    meq[M11] = 0.0;                                  /* equilibria, Tab. scheme */
    meq[MS] = 0.0;
    meq[MD] = 0.0;
    meq[M12] = theta * mb10;
    meq[M21] = theta * mb01;
    meq[M22] = 0.0;
    for (int a = M11; a <= M22; ++a)                 /* relax (Eq. collision)  */
        mstar[a] = omega[a] * meq[a] + (1.0 - omega[a]) * m[a];
    mstar[M10] = mb10 + 0.5 * gx;                    /* half forcing (post)    */
    mstar[M01] = mb01 + 0.5 * gy;
    for (int i = 0; i < 8; ++i) {                    /* back-transformation    */
        double s = 0.0;
        for (int j = 0; j < 8; ++j) s += g_Minv[i][j] * mstar[j];
        fstar[i] = s;
    }
}

/* ---------------------------------------------------------------------- */
/* Lattice-wide passes                                                     */
/* ---------------------------------------------------------------------- */

static inline long pidx(int nx, int ny, int q, int x, int y) {
    return (long)q * nx * ny + (long)y * nx + x;
}

static inline int wrap(int i, int n) {
    int r = i % n;
    return r < 0 ? r + n : r;
}

/* Collide every node of f into fstar (separate arrays). */
void oracle_collide_all(int nx, int ny, const double *f, const double *gx, const double *gy,
                        const double omega[8], double theta, double *fstar) {
    build_transform();
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            double fl[8], fs[8];
            long s = (long)y * nx + x;
            for (int q = 0; q < 8; ++q) fl[q] = f[pidx(nx, ny, q, x, y)];
            oracle_collide_node(fl, gx[s], gy[s], omega, theta, fs, NULL);
            for (int q = 0; q < 8; ++q) fstar[pidx(nx, ny, q, x, y)] = fs[q];
        }
    }
}

/* Streaming (Eq. streaming) with periodic wrap: the population leaving node
 * x along c_q arrives at (x + c_q) mod (nx, ny). */
void oracle_stream(int nx, int ny, const double *fstar, double *fnext) {
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x)
            for (int q = 0; q < 8; ++q) {
                int xd = wrap(x + CX[q], nx), yd = wrap(y + CY[q], ny);
                fnext[pidx(nx, ny, q, xd, yd)] = fstar[pidx(nx, ny, q, x, y)];
            }
}

/* Advance the state f (pre-collision populations f(n)) by nsteps steps of
 * Algorithm 1, in place.  Returns 0, or -1 on allocation failure. */
int oracle_run(int nx, int ny, double *f, const double *gx, const double *gy,
               const double omega[8], double theta, long nsteps) {
    size_t n = (size_t)8 * nx * ny;
    double *fs = (double *)malloc(n * sizeof(double));
    if (!fs) return -1;
    for (long k = 0; k < nsteps; ++k) {
        oracle_collide_all(nx, ny, f, gx, gy, omega, theta, fs);
        oracle_stream(nx, ny, fs, f);
    }
    free(fs);
    return 0;
}

/* Displacement u(n) = (m10 + gx/2, m01 + gy/2) of the state f(n)
 * (Table "solution", Eqs. coll10/coll01). */
void oracle_displacement(int nx, int ny, const double *f, const double *gx, const double *gy,
                         double *ux, double *uy) {
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double fl[8];
            long s = (long)y * nx + x;
            for (int q = 0; q < 8; ++q) fl[q] = f[pidx(nx, ny, q, x, y)];
            ux[s] = raw_moment(fl, 1, 0) + 0.5 * gx[s];
            uy[s] = raw_moment(fl, 0, 1) + 0.5 * gy[s];
        }
}

/* Stress of the state f(n) in lattice units from the bared second-order
 * moments (Eq. compute_bared with m_eq = 0 for 11, s, d; Table "solution"
 * without the 1/eps factor): sxx = -(mb_s + mb_d)/2, syy = -(mb_s - mb_d)/2,
 * sxy = -mb_11. */
void oracle_stress(int nx, int ny, const double *f, const double omega[8], double *sxx,
                   double *syy, double *sxy) {
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double fl[8], m[8];
            long s = (long)y * nx + x;
            for (int q = 0; q < 8; ++q) fl[q] = f[pidx(nx, ny, q, x, y)];
            moments(fl, m);
            /* bared moment: (omega/2) m_eq + (1 - omega/2) m, with m_eq = 0 */
            double mb11 = (1.0 - 0.5 * omega[M11]) * m[M11];
            double mbs = (1.0 - 0.5 * omega[MS]) * m[MS];
            double mbd = (1.0 - 0.5 * omega[MD]) * m[MD];
            sxx[s] = -0.5 * (mbs + mbd);
            syy[s] = -0.5 * (mbs - mbd);
            sxy[s] = -mb11;
        }
}

/* Steady-state residual r = ||u - u_prev||_2 / ||u||_2 summed over all nodes
 * and both components (the grid spacing cancels); 0 if both norms are 0.
 * The paper asks for ||d_t u|| < TOL "in some norm" (Sec. 2.1); this is the
 * L2 grid norm of Sec. 7.1 taken as a ratio. */
double oracle_residual(long n, const double *ux, const double *uy, const double *uxp,
                       const double *uyp) {
    double d = 0.0, s = 0.0;
    for (long i = 0; i < n; ++i) {
        double dx = ux[i] - uxp[i], dy = uy[i] - uyp[i];
        d += dx * dx + dy * dy;
        s += ux[i] * ux[i] + uy[i] * uy[i];
    }
    if (s == 0.0) return d == 0.0 ? 0.0 : INFINITY;
    return sqrt(d / s);
}

/* Pseudo-time stepping to steady state: step; at n = K, 2K, ... evaluate
 * r(n) = ||u(n) - u(n-1)|| / ||u(n)|| and stop at the first n with
 * r(n) <= tol, or when n reaches max_steps.  f holds f(n) on return.
 * *steps_out = n, *r_out = last residual evaluated (NAN if none).
 * Returns 0 on convergence, 1 if max_steps was reached, -1 on allocation
 * failure, -2 on divergence: a non-finite residual, or (rise_checks > 0) an
 * update norm d(n) = ||u(n) - u(n-1)||_2 (the residual's numerator) that rose
 * at each of rise_checks checks in a row and is at least twice the largest of
 * the 32 update norms before those rises.  The paper gives no divergence rule;
 * the rise rule is the solve's stop policy for materials outside the stable
 * region of Sec. 5, checked after the tolerance and the step limit.  (Under an
 * instability d grows geometrically without end, while r saturates once the
 * unstable modes dominate u; a decaying oscillation makes d climb from its
 * dips for several checks, but never above its earlier peaks.) */
int oracle_solve_to_tol(int nx, int ny, double *f, const double *gx, const double *gy,
                        const double omega[8], double theta, double tol, long max_steps,
                        int check_every, int rise_checks, long *steps_out, double *r_out) {
    long ns = (long)nx * ny;
    double *fs = (double *)malloc((size_t)8 * ns * sizeof(double));
    double *u = (double *)malloc((size_t)4 * ns * sizeof(double));
    if (!fs || !u) { free(fs); free(u); return -1; }
    double *ux = u, *uy = u + ns, *uxp = u + 2 * ns, *uyp = u + 3 * ns;
    if (check_every < 1) check_every = 1;
    long n = 0;
    int status = 1;
    double d_prev = NAN, d_before_rises = NAN;
    double hist[32];
    int rises = 0, nhist = 0;
    *r_out = NAN;
    while (n < max_steps) {
        if ((n + 1) % check_every == 0)
            oracle_displacement(nx, ny, f, gx, gy, uxp, uyp); /* u(n) before stepping */
        oracle_collide_all(nx, ny, f, gx, gy, omega, theta, fs);
        oracle_stream(nx, ny, fs, f);
        ++n;
        if (n % check_every == 0) {
            oracle_displacement(nx, ny, f, gx, gy, ux, uy);
            double r = oracle_residual(ns, ux, uy, uxp, uyp);
            *r_out = r;
            if (!isfinite(r)) { status = -2; break; }
            if (r <= tol) { status = 0; break; }
            if (n >= max_steps) break;
            double d = 0.0;
            for (long i = 0; i < ns; ++i) {
                double ex = ux[i] - uxp[i], ey = uy[i] - uyp[i];
                d += ex * ex + ey * ey;
            }
            d = sqrt(d);
            if (d > d_prev) {
                if (rises == 0) {
                    d_before_rises = hist[0];
                    for (int h = 1; h < nhist && h < 32; ++h)
                        if (hist[h] > d_before_rises) d_before_rises = hist[h];
                }
                ++rises;
            } else {
                rises = 0;
            }
            hist[nhist % 32] = d;
            ++nhist;
            d_prev = d;
            if (rise_checks > 0 && rises >= rise_checks && d >= 2.0 * d_before_rises) {
                status = -2;
                break;
            }
        }
    }
    *steps_out = n;
    free(fs);
    free(u);
    return status;
}

/* Streaming alone (no collision) for nsteps steps, in place: the bit-exact
 * reference for the index arithmetic of the GPU kernels. */
int oracle_stream_only(int nx, int ny, double *f, long nsteps) {
    size_t n = (size_t)8 * nx * ny;
    double *tmp = (double *)malloc(n * sizeof(double));
    if (!tmp) return -1;
    for (long k = 0; k < nsteps; ++k) {
        memcpy(tmp, f, n * sizeof(double));
        oracle_stream(nx, ny, tmp, f);
    }
    free(tmp);
    return 0;
}
