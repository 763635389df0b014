/*
 * ORACLE -- test infrastructure only.  Plain, slow, FP64 reference of the
 * rigid-body pair path.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library; the product path never does.
 *
 * Conventions: quaternions q = (w, x, y, z), Hamilton product, unit norm,
 * R(q) maps body-frame vectors to the lab frame.  Bead templates are given in
 * the body frame with the centre of mass at the origin.  Positions,
 * orientations and momenta are arrays of structures: x[3*i+a], q[4*i+c].
 *
 * Contents
 *   oracle_lj                 bead-bead Lennard-Jones 12-6, energy-shifted
 *   oracle_hphc               bead-bead half-power half-cosine potential
 *                             (paper section 3), selected for all the sums
 *                             below by oracle_set_hphc (oracle_set_lj: back)
 *   oracle_bead_pair          double sum over the beads of two bodies
 *                             (paper section 2, first equation)
 *   oracle_bead_system        that double sum for every pair of bodies whose
 *                             centres are close enough for any bead pair to
 *                             be inside the cutoff, accumulated per body
 *   oracle_pairs_within       brute-force list of body pairs within a radius
 *   oracle_rigid_phase1/2     rigid-body velocity Verlet with the NO_SQUISH
 *                             free-rotation splitting (Miller, Eleftheriou,
 *                             Pattnaik, Ndirango, Newns, Martyna, J. Chem.
 *                             Phys. 116, 8649 (2002)); the paper fixes only
 *                             the time step (section 3, dt = 0.005 tau)
 *   oracle_nve                NVE run driving the two phases with bead forces
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double kPi = 3.14159265358979323846;

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------- algebra */

static void qmat(const double *q, double R[3][3]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0][0] = 1 - 2 * (y * y + z * z); R[0][1] = 2 * (x * y - w * z); R[0][2] = 2 * (x * z + w * y);
    R[1][0] = 2 * (x * y + w * z); R[1][1] = 1 - 2 * (x * x + z * z); R[1][2] = 2 * (y * z - w * x);
    R[2][0] = 2 * (x * z - w * y); R[2][1] = 2 * (y * z + w * x); R[2][2] = 1 - 2 * (x * x + y * y);
}

static void matvec(double R[3][3], const double *v, double *o) {
    for (int a = 0; a < 3; ++a) o[a] = R[a][0] * v[0] + R[a][1] * v[1] + R[a][2] * v[2];
}

static void matTvec(double R[3][3], const double *v, double *o) {
    for (int a = 0; a < 3; ++a) o[a] = R[0][a] * v[0] + R[1][a] * v[1] + R[2][a] * v[2];
}

static void cross(const double *a, const double *b, double *o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

/* Hamilton product o = a * b. */
static void qmul(const double *a, const double *b, double *o) {
    double r[4];
    r[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    r[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    r[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    r[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
    memcpy(o, r, sizeof r);
}

static void min_image(double *d, const double *box) {
    if (!box) return;
    for (int a = 0; a < 3; ++a) d[a] -= box[a] * nearbyint(d[a] / box[a]);
}

/* ------------------------------------------------------------- bead pair */

/* Lennard-Jones 12-6 between two beads at squared distance r2, cut at rc and
 * shifted in energy only: u(r) - u(rc) for r < rc, 0 beyond.  Returns the
 * energy and writes -(du/dr)/r, so the force on the first bead is
 * (*f_over_r) * (r_1 - r_2). */
double oracle_lj(double r2, double eps, double sigma, double rc, double *f_over_r) {
    if (r2 >= rc * rc) { *f_over_r = 0.0; return 0.0; }
    double s2 = sigma * sigma / r2, s6 = s2 * s2 * s2, s12 = s6 * s6;
    double sc = sigma / rc, sc6 = pow(sc, 6), sc12 = sc6 * sc6;
    *f_over_r = 24.0 * eps * (2.0 * s12 - s6) / r2;
    return 4.0 * eps * (s12 - s6) - 4.0 * eps * (sc12 - sc6);
}

/* Half-power half-cosine potential (paper section 3): a soft repulsion
 * (b - r)^p - 2A for r <= b and a cosine well beyond.  The printed attractive
 * branch, -A cos(c (r - b)), would jump from -2A to -A at r = b and end at +A
 * at the end of the half period; it is read here as -A (1 + cos(c (r - b))),
 * which joins the repulsive branch at r = b with zero slope and reaches zero
 * with zero slope at r_c = b + pi / c, the cutoff.  Returns the energy and
 * writes -(dU/dr)/r. */
double oracle_hphc(double r2, double A, double b, double c, double p, double *f_over_r) {
    const double rcut = b + kPi / c;
    if (r2 >= rcut * rcut) { *f_over_r = 0.0; return 0.0; }
    const double r = sqrt(r2);
    if (r <= b) {
        const double t = b - r;
        *f_over_r = p * pow(t, p - 1.0) / r;
        return pow(t, p) - 2.0 * A;
    }
    const double x = c * (r - b);
    *f_over_r = -A * c * sin(x) / r;
    return -A * (1.0 + cos(x));
}

/* Bead potential used by the sums: 0 = Lennard-Jones (eps, sigma, rc passed
 * in), 1 = half-power half-cosine with the parameters set here. */
static int g_pot = 0;
static double g_hphc[4];

void oracle_set_hphc(double A, double b, double c, double p) {
    g_pot = 1;
    g_hphc[0] = A; g_hphc[1] = b; g_hphc[2] = c; g_hphc[3] = p;
}

void oracle_set_lj(void) { g_pot = 0; }

static double bead_cutoff(double rc) { return g_pot ? g_hphc[1] + kPi / g_hphc[2] : rc; }

static double bead_u(double r2, double eps, double sigma, double rc, double *f_over_r) {
    if (g_pot) return oracle_hphc(r2, g_hphc[0], g_hphc[1], g_hphc[2], g_hphc[3], f_over_r);
    return oracle_lj(r2, eps, sigma, rc, f_over_r);
}

/* Energy, forces and torques between body i and body j: the sum of the bead
 * interaction over all N_i x N_j bead pairs (paper section 2).  Every bead
 * force is accumulated directly into both bodies; torques are about each
 * body's own centre.  box == NULL means no periodic images.
 * out[14] = E, F_i[3], F_j[3], tau_i[3], tau_j[3], r_min (over all pairs). */
void oracle_bead_pair(int ni, const double *bi, int nj, const double *bj,
                      const double *xi, const double *qi, const double *xj, const double *qj,
                      const double *box, double eps, double sigma, double rc, double *out) {
    double Ri[3][3], Rj[3][3], dlab[3];
    const double rcut = bead_cutoff(rc);
    qmat(qi, Ri); qmat(qj, Rj);
    for (int a = 0; a < 3; ++a) dlab[a] = xj[a] - xi[a];
    min_image(dlab, box);
    double E = 0, Fi[3] = {0, 0, 0}, Fj[3] = {0, 0, 0}, Ti[3] = {0, 0, 0}, Tj[3] = {0, 0, 0};
    double rmin2 = INFINITY;
    double *rl = (double *)malloc(sizeof(double) * 3 * (size_t)nj);
    for (int l = 0; l < nj; ++l) matvec(Rj, bj + 3 * l, rl + 3 * l);   /* relative to x_j */
    for (int k = 0; k < ni; ++k) {
        double rk[3];
        matvec(Ri, bi + 3 * k, rk);                                      /* relative to x_i */
        for (int l = 0; l < nj; ++l) {
            double v[3], r2 = 0, fr, f[3], t[3], lj[3];
            for (int a = 0; a < 3; ++a) {
                lj[a] = dlab[a] + rl[3 * l + a];                         /* bead l relative to x_i */
                v[a] = rk[a] - lj[a];
                r2 += v[a] * v[a];
            }
            if (r2 < rmin2) rmin2 = r2;
            if (r2 >= rcut * rcut) continue;
            E += bead_u(r2, eps, sigma, rc, &fr);
            for (int a = 0; a < 3; ++a) f[a] = fr * v[a];                /* force on bead k */
            for (int a = 0; a < 3; ++a) { Fi[a] += f[a]; Fj[a] -= f[a]; }
            cross(rk, f, t);
            for (int a = 0; a < 3; ++a) Ti[a] += t[a];
            double mf[3] = {-f[0], -f[1], -f[2]};
            cross(rl + 3 * l, mf, t);                                    /* arm about x_j */
            for (int a = 0; a < 3; ++a) Tj[a] += t[a];
        }
    }
    free(rl);
    out[0] = E;
    for (int a = 0; a < 3; ++a) {
        out[1 + a] = Fi[a]; out[4 + a] = Fj[a]; out[7 + a] = Ti[a]; out[10 + a] = Tj[a];
    }
    out[13] = sqrt(rmin2);
}

/* Body pairs (i < j) whose minimum-image centre distance is below r, by
 * testing all n(n-1)/2 pairs.  Writes at most max_pairs pairs; returns the
 * total number found. */
long oracle_pairs_within(int n, const double *x, const double *box, double r,
                         long max_pairs, int *pi, int *pj) {
    long cnt = 0;
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            double d[3];
            for (int a = 0; a < 3; ++a) d[a] = x[3 * j + a] - x[3 * i + a];
            min_image(d, box);
            if (d[0] * d[0] + d[1] * d[1] + d[2] * d[2] < r * r) {
                if (cnt < max_pairs) { pi[cnt] = i; pj[cnt] = j; }
                ++cnt;
            }
        }
    return cnt;
}

static double template_rmax(int n, const double *b) {
    double m = 0;
    for (int k = 0; k < n; ++k) {
        double r2 = b[3 * k] * b[3 * k] + b[3 * k + 1] * b[3 * k + 1] + b[3 * k + 2] * b[3 * k + 2];
        if (r2 > m) m = r2;
    }
    return sqrt(m);
}

/* Total energy, per-body force and torque, and the molecular virial
 * W_ab = sum over pairs of d_a F_j,b (d = x_j - x_i, minimum image, F_j the
 * force on j) for a periodic system of rigid bodies.  A pair can only have
 * bead pairs inside rc when its centre distance is below
 * rmax_i + rmax_j + rc (triangle inequality), so only those pairs are summed.
 * Templates of all types are concatenated in `tmpl`, type t starting at bead
 * offset off[t] with nb[t] beads.  Returns the number of pairs summed. */
long oracle_bead_system(int n, const double *x, const double *q, const int *type,
                        int ntypes, const int *nb, const int *off, const double *tmpl,
                        const double *box, double eps, double sigma, double rc,
                        double *energy, double *force, double *torque, double *virial) {
    double *rmax = (double *)malloc(sizeof(double) * (size_t)ntypes);
    for (int t = 0; t < ntypes; ++t) rmax[t] = template_rmax(nb[t], tmpl + 3 * (size_t)off[t]);
    long cap = 1024, np = 0;
    int *pi = (int *)malloc(sizeof(int) * cap), *pj = (int *)malloc(sizeof(int) * cap);
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            double d[3];
            for (int a = 0; a < 3; ++a) d[a] = x[3 * j + a] - x[3 * i + a];
            min_image(d, box);
            double c = rmax[type[i]] + rmax[type[j]] + bead_cutoff(rc);
            if (d[0] * d[0] + d[1] * d[1] + d[2] * d[2] >= c * c) continue;
            if (np == cap) {
                cap *= 2;
                pi = (int *)realloc(pi, sizeof(int) * cap);
                pj = (int *)realloc(pj, sizeof(int) * cap);
            }
            pi[np] = i; pj[np] = j; ++np;
        }
    double *res = (double *)malloc(sizeof(double) * 14 * (size_t)(np ? np : 1));
#pragma omp parallel for schedule(dynamic, 4)
    for (long p = 0; p < np; ++p) {
        int i = pi[p], j = pj[p];
        oracle_bead_pair(nb[type[i]], tmpl + 3 * (size_t)off[type[i]], nb[type[j]],
                         tmpl + 3 * (size_t)off[type[j]], x + 3 * i, q + 4 * i, x + 3 * j, q + 4 * j,
                         box, eps, sigma, rc, res + 14 * p);
    }
    memset(force, 0, sizeof(double) * 3 * n);
    memset(torque, 0, sizeof(double) * 3 * n);
    memset(virial, 0, sizeof(double) * 9);
    double E = 0;
    for (long p = 0; p < np; ++p) {
        const double *r = res + 14 * p;
        int i = pi[p], j = pj[p];
        double d[3];
        for (int a = 0; a < 3; ++a) d[a] = x[3 * j + a] - x[3 * i + a];
        min_image(d, box);
        E += r[0];
        for (int a = 0; a < 3; ++a) {
            force[3 * i + a] += r[1 + a]; force[3 * j + a] += r[4 + a];
            torque[3 * i + a] += r[7 + a]; torque[3 * j + a] += r[10 + a];
            for (int b = 0; b < 3; ++b) virial[3 * a + b] += d[a] * r[4 + b];
        }
    }
    *energy = E;
    free(res); free(pi); free(pj); free(rmax);
    return np;
}

/* ------------------------------------------------------------- integrator */

/* NO_SQUISH: the rotational state is (q, p) with p = 2 S(q) (0, L_body)
 * = 2 q * (0, L) the conjugate quaternion momentum.  P_k q = q * e_k for the
 * quaternion units e_1 = i, e_2 = j, e_3 = k.  The free-rotation flow of the
 * k-th term of the kinetic energy, (p . P_k q)^2 / (8 I_k), over a time h
 * rotates (q, p) in the planes (q, P_k q), (p, P_k p) by the angle
 * zeta = h (p . P_k q) / (4 I_k). */
static void perm_k(int k, const double *v, double *o) {
    double e[4] = {0, 0, 0, 0};
    e[k] = 1.0;
    qmul(v, e, o);
}

static void free_rot_k(int k, double h, double I, double *q, double *p) {
    double Pq[4], Pp[4];
    perm_k(k, q, Pq);
    perm_k(k, p, Pp);
    double s = p[0] * Pq[0] + p[1] * Pq[1] + p[2] * Pq[2] + p[3] * Pq[3];
    double zeta = h * s / (4.0 * I);
    double c = cos(zeta), sn = sin(zeta);
    for (int a = 0; a < 4; ++a) {
        q[a] = c * q[a] + sn * Pq[a];
        p[a] = c * p[a] + sn * Pp[a];
    }
}

static void L_to_p(const double *q, const double *L, double *p) {
    double l4[4] = {0, L[0], L[1], L[2]};
    qmul(q, l4, p);
    for (int a = 0; a < 4; ++a) p[a] *= 2.0;
}

static void p_to_L(const double *q, const double *p, double *L) {
    double qc[4] = {q[0], -q[1], -q[2], -q[3]}, r[4];
    qmul(qc, p, r);
    L[0] = 0.5 * r[1]; L[1] = 0.5 * r[2]; L[2] = 0.5 * r[3];
}

/* Half kick with the body-frame torque: dL_body = (dt/2) R(q)^T tau_lab
 * (equivalently dp = dt S(q)(0, tau_body)); dP = (dt/2) F. */
static void half_kick(double dt, double *P, const double *q, double *L, const double *F,
                      const double *tau) {
    double R[3][3], tb[3];
    qmat(q, R);
    matTvec(R, tau, tb);
    for (int a = 0; a < 3; ++a) { P[a] += 0.5 * dt * F[a]; L[a] += 0.5 * dt * tb[a]; }
}

/* Phase 1 of a step for every body: half kick, drift x += dt P / M, free
 * rotation R3(dt/2) R2(dt/2) R1(dt) R2(dt/2) R3(dt/2), renormalise q.
 * mass[i] and inertia[3i+a] are per body. */
void oracle_rigid_phase1(int n, double dt, double *x, double *P, double *q, double *L,
                         const double *mass, const double *inertia, const double *F,
                         const double *tau) {
    for (int i = 0; i < n; ++i) {
        half_kick(dt, P + 3 * i, q + 4 * i, L + 3 * i, F + 3 * i, tau + 3 * i);
        for (int a = 0; a < 3; ++a) x[3 * i + a] += dt * P[3 * i + a] / mass[i];
        double p[4], *qi = q + 4 * i;
        const double *I = inertia + 3 * i;
        L_to_p(qi, L + 3 * i, p);
        free_rot_k(3, 0.5 * dt, I[2], qi, p);
        free_rot_k(2, 0.5 * dt, I[1], qi, p);
        free_rot_k(1, dt, I[0], qi, p);
        free_rot_k(2, 0.5 * dt, I[1], qi, p);
        free_rot_k(3, 0.5 * dt, I[2], qi, p);
        double nq = sqrt(qi[0] * qi[0] + qi[1] * qi[1] + qi[2] * qi[2] + qi[3] * qi[3]);
        for (int a = 0; a < 4; ++a) qi[a] /= nq;
        p_to_L(qi, p, L + 3 * i);
    }
}

/* Phase 2: the second half kick with the new forces.  Returns the kinetic
 * energy sum P^2/(2M) + sum_a L_a^2/(2 I_a). */
double oracle_rigid_phase2(int n, double dt, double *P, const double *q, double *L,
                           const double *mass, const double *inertia, const double *F,
                           const double *tau) {
    double ke = 0;
    for (int i = 0; i < n; ++i) {
        half_kick(dt, P + 3 * i, q + 4 * i, L + 3 * i, F + 3 * i, tau + 3 * i);
        for (int a = 0; a < 3; ++a) {
            ke += P[3 * i + a] * P[3 * i + a] / (2.0 * mass[i]);
            ke += L[3 * i + a] * L[3 * i + a] / (2.0 * inertia[3 * i + a]);
        }
    }
    return ke;
}

/* NVE run with bead forces: force evaluation at the start, then `steps`
 * velocity-Verlet steps.  pe[s], ke[s] receive the potential and kinetic
 * energy after step s (s = 0 is the initial state, arrays of steps+1). */
void oracle_nve(int n, int steps, double dt, double *x, double *P, double *q, double *L,
                const int *type, const double *mass_t, const double *inertia_t, int ntypes,
                const int *nb, const int *off, const double *tmpl, const double *box,
                double eps, double sigma, double rc, double *pe, double *ke) {
    double *F = (double *)malloc(sizeof(double) * 3 * n), *T = (double *)malloc(sizeof(double) * 3 * n);
    double *m = (double *)malloc(sizeof(double) * n), *I = (double *)malloc(sizeof(double) * 3 * n);
    double W[9];
    for (int i = 0; i < n; ++i) {
        m[i] = mass_t[type[i]];
        for (int a = 0; a < 3; ++a) I[3 * i + a] = inertia_t[3 * type[i] + a];
    }
    oracle_bead_system(n, x, q, type, ntypes, nb, off, tmpl, box, eps, sigma, rc, pe, F, T, W);
    double k0 = 0;
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a)
            k0 += P[3 * i + a] * P[3 * i + a] / (2 * m[i]) + L[3 * i + a] * L[3 * i + a] / (2 * I[3 * i + a]);
    ke[0] = k0;
    for (int s = 1; s <= steps; ++s) {
        oracle_rigid_phase1(n, dt, x, P, q, L, m, I, F, T);
        oracle_bead_system(n, x, q, type, ntypes, nb, off, tmpl, box, eps, sigma, rc, pe + s, F, T, W);
        ke[s] = oracle_rigid_phase2(n, dt, P, q, L, m, I, F, T);
    }
    free(F); free(T); free(m); free(I);
}
