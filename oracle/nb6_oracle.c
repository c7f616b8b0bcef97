/*
 * nb6_oracle.c -- FP64 CPU oracle for the regular and irregular forces of the
 * Ahmad-Cohen neighbour scheme (Nitadori & Aarseth 2012, "Accelerating NBODY6 with
 * Graphics Processing Units").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference that the GPU library
 * is checked against.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header or
 * constant with the HIP library, and the library never calls it.
 *
 * Everything is plain IEEE double precision, written as the definitions in
 * the paper state them, without blocking or reordering:
 *
 *   - nb6o_predict: the cubic Taylor predictor of positions and velocities
 *     to the block time, built from the stored position, velocity,
 *     acceleration and jerk (section 3.3, step 3, "predict all particles
 *     needed"; the host routine that predicts all particles in Appendix C,
 *     Listing C1).
 *
 *   - nb6o_regular_force: for each active i and every j != i, the velocity
 *     neighbour criterion of section 3.2 (the smaller of the two end-point
 *     distances |R_ij| and |R_ij + dt_reg,i V_ij| compared with h_i), then
 *     the regular force and its time derivative of section 3.3, step 6
 *     (the F_reg and dF_reg/dt sums over non-neighbours), the neighbour
 *     list L_i of the same step, and optionally the regular potential (the
 *     extra sum the appendix kernel adds under its POTENTIAL switch; section
 *     4 quotes its accuracy for the energy check).
 *
 *   - nb6o_pair_terms: the same pair quantities for an explicit list of
 *     (i, j) pairs; the tests use it to treat pairs that sit on the
 *     neighbour-radius boundary.
 *
 *   - nb6o_regular_correct: the regular corrector of a block -- the
 *     neighbour-change correction of the regular force difference (section
 *     3.6), the derivatives of the regular force by Hermite interpolation,
 *     the next regular step and the new neighbour radius (equation 1).
 *
 *   - nb6o_irregular_force: the irregular force and its time derivative of
 *     section 3.3 step 4, the sums over the entries of each active
 *     particle's neighbour list L_i (the quantity the irregular-force
 *     library of section 3.5 returns for a list of active particles).
 *
 * Readings of the paper taken here (each is listed with its reason in the
 * design notes of the repository):
 *   - R_ij = R_j - R_i and V_ij = V_j - V_i (section 3.2), G = 1.
 *   - The neighbour test is strict: j is a neighbour iff
 *     min(|R|^2, |R + dtr V|^2) < h^2.  Equality contributes force.  The two
 *     force cases of section 3.3 are written with "> h" and the list with
 *     "< h"; the appendix kernel (Listing B2) uses the strict "<" for the
 *     list and adds force otherwise, which is the exact partition used here.
 *   - Only the two end points of the interval enter the criterion
 *     (section 3.2), not the closest approach between them.
 *   - j = i is excluded by index; it is never a neighbour and never a term.
 *   - Lists are returned in ascending j (section 3.6 relies on the
 *     sequential ordering of neighbour lists).
 *   - h^2 must be > 0.
 *
 * Sums over j use Neumaier's compensated summation in FP64 so that the
 * oracle's own rounding error (~1e-16 relative to the sum of |terms|) is far
 * below the 1e-6 tolerance of the checks that use it.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------------- */
/* Neumaier compensated accumulator                                        */
/* ---------------------------------------------------------------------- */
typedef struct { double s, c; } nsum;

static void nsum_add(nsum *a, double t)
{
    double s = a->s + t;
    if (fabs(a->s) >= fabs(t))
        a->c += (a->s - s) + t;
    else
        a->c += (t - s) + a->s;
    a->s = s;
}

static double nsum_get(const nsum *a) { return a->s + a->c; }

/* ---------------------------------------------------------------------- */
/* Prediction (section 3.3 step 3; Appendix C predictor call)              */
/* ---------------------------------------------------------------------- */
/*
 * For every particle k: dt = tb - t[k];
 *   xp = x + v dt + a dt^2/2 + jerk dt^3/6
 *   vp = v + a dt + jerk dt^2/2
 * Arrays x, v, a, jerk, xp, vp are [n][3]; t is [n].
 */
void nb6o_predict(int64_t n, const double *x, const double *v,
                  const double *a, const double *jerk, const double *t,
                  double tb, double *xp, double *vp)
{
    for (int64_t k = 0; k < n; ++k) {
        double dt = tb - t[k];
        for (int c = 0; c < 3; ++c) {
            int64_t q = 3 * k + c;
            xp[q] = x[q] + v[q] * dt + a[q] * dt * dt / 2.0
                  + jerk[q] * dt * dt * dt / 6.0;
            vp[q] = v[q] + a[q] * dt + jerk[q] * dt * dt / 2.0;
        }
    }
}

/* ---------------------------------------------------------------------- */
/* Regular force, jerk and neighbour list (sections 3.2 and 3.3 step 6)    */
/* ---------------------------------------------------------------------- */
/*
 * Inputs
 *   n            number of j-particles (the whole cluster)
 *   m[n], xp[n][3], vp[n][3]  predicted j state
 *   ni           number of active i-particles
 *   idx[ni]      indices of the active particles (0 <= idx < n)
 *   h2[ni]       squared neighbour radius of each active particle (> 0)
 *   dtr[ni]      regular time-step of each active particle
 *   lcap         capacity of each row of `list`
 *   nthreads     OpenMP threads (<= 0: library default)
 * Outputs
 *   acc[ni][3], jrk[ni][3]  regular force and its time derivative
 *   nnb[ni]      true neighbour count
 *   list[ni][lcap]  first min(nnb, lcap) neighbours, ascending j
 *   sa[ni]       sum over non-neighbours of m_j / r^2        (may be NULL)
 *   sj[ni]       sum over non-neighbours of
 *                m_j (|V|/r^3 + 3 |R.V| / r^4)               (may be NULL)
 *   pot[ni]      regular potential, -sum over non-neighbours of m_j / r
 *                (the optional potential sum of the appendix kernel, with
 *                the physical sign)                          (may be NULL)
 * Returns 0, or -1 for a bad index, -2 for h2 <= 0 (nothing is computed
 * for that i).
 */
int nb6o_regular_force(int64_t n, const double *m, const double *xp,
                       const double *vp, int64_t ni, const int32_t *idx,
                       const double *h2, const double *dtr,
                       double *acc, double *jrk, int32_t *nnb,
                       int32_t *list, int64_t lcap,
                       double *sa, double *sj, double *pot, int nthreads)
{
    for (int64_t q = 0; q < ni; ++q) {
        if (idx[q] < 0 || idx[q] >= n) return -1;
        if (!(h2[q] > 0.0)) return -2;
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif

#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < ni; ++q) {
        const int64_t i = idx[q];
        const double hi2 = h2[q];
        const double dti = dtr[q];
        nsum A[3] = {{0, 0}, {0, 0}, {0, 0}};
        nsum J[3] = {{0, 0}, {0, 0}, {0, 0}};
        nsum SA = {0, 0}, SJ = {0, 0}, PHI = {0, 0};
        int64_t count = 0;

        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double R[3], V[3], P[3];
            for (int c = 0; c < 3; ++c) {
                R[c] = xp[3 * j + c] - xp[3 * i + c];
                V[c] = vp[3 * j + c] - vp[3 * i + c];
                P[c] = R[c] + dti * V[c];
            }
            double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
            double p2 = P[0] * P[0] + P[1] * P[1] + P[2] * P[2];
            double rmin2 = (p2 < r2) ? p2 : r2;

            if (rmin2 < hi2) {
                /* neighbour: listed, no regular force */
                if (count < lcap) list[q * lcap + count] = (int32_t)j;
                ++count;
                continue;
            }
            double r = sqrt(r2);
            double r3 = r2 * r;
            double r5 = r3 * r2;
            double rv = R[0] * V[0] + R[1] * V[1] + R[2] * V[2];
            for (int c = 0; c < 3; ++c) {
                nsum_add(&A[c], m[j] * R[c] / r3);
                nsum_add(&J[c], m[j] * (V[c] / r3 - 3.0 * rv * R[c] / r5));
            }
            double vabs = sqrt(V[0] * V[0] + V[1] * V[1] + V[2] * V[2]);
            nsum_add(&SA, m[j] / r2);
            nsum_add(&SJ, m[j] * (vabs / r3 + 3.0 * fabs(rv) / (r2 * r2)));
            nsum_add(&PHI, -m[j] / r);
        }
        for (int c = 0; c < 3; ++c) {
            acc[3 * q + c] = nsum_get(&A[c]);
            jrk[3 * q + c] = nsum_get(&J[c]);
        }
        nnb[q] = (int32_t)count;
        if (sa) sa[q] = nsum_get(&SA);
        if (sj) sj[q] = nsum_get(&SJ);
        if (pot) pot[q] = nsum_get(&PHI);
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Per-pair quantities for an explicit list of pairs                       */
/* ---------------------------------------------------------------------- */
/*
 * For pair p (i = pi[p], j = pj[p], time-step dtr[p]):
 *   rmin[p]     = sqrt(min(|R|^2, |R + dtr V|^2))
 *   dacc[p][3]  = m_j R / r^3
 *   djrk[p][3]  = m_j (V / r^3 - 3 (R.V) R / r^5)
 * i.e. the contribution the pair makes to the regular sums when it is not a
 * neighbour.  Used to move boundary pairs between the neighbour list and the
 * force sum.
 */
void nb6o_pair_terms(int64_t np, const int32_t *pi, const int32_t *pj,
                     const double *dtr, const double *m, const double *xp,
                     const double *vp, double *rmin, double *dacc,
                     double *djrk)
{
    for (int64_t p = 0; p < np; ++p) {
        int64_t i = pi[p], j = pj[p];
        double R[3], V[3], P[3];
        for (int c = 0; c < 3; ++c) {
            R[c] = xp[3 * j + c] - xp[3 * i + c];
            V[c] = vp[3 * j + c] - vp[3 * i + c];
            P[c] = R[c] + dtr[p] * V[c];
        }
        double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
        double p2 = P[0] * P[0] + P[1] * P[1] + P[2] * P[2];
        rmin[p] = sqrt((p2 < r2) ? p2 : r2);
        double r = sqrt(r2);
        double r3 = r2 * r;
        double r5 = r3 * r2;
        double rv = R[0] * V[0] + R[1] * V[1] + R[2] * V[2];
        for (int c = 0; c < 3; ++c) {
            dacc[3 * p + c] = m[j] * R[c] / r3;
            djrk[3 * p + c] = m[j] * (V[c] / r3 - 3.0 * rv * R[c] / r5);
        }
    }
}

/* ---------------------------------------------------------------------- */
/* Irregular force and its derivative over neighbour lists                 */
/* (section 3.3 step 4; the irregular-force library of section 3.5)        */
/* ---------------------------------------------------------------------- */
/*
 * For each active i = idx[q] and every entry j of its list L_i:
 *   F_I,i  = sum_{j in L_i} m_j R_ij / |R_ij|^3
 *   dF_I,i = sum_{j in L_i} m_j (V_ij / |R_ij|^3
 *                                - 3 (R_ij . V_ij) R_ij / |R_ij|^5)
 * with R_ij = R_j - R_i and V_ij = V_j - V_i of the predicted state.
 * Inputs
 *   n, m[n], xp[n][3], vp[n][3]   predicted state of the cluster
 *   ni, idx[ni]                   active particles (0 <= idx < n)
 *   cnt[ni]                       entries of each list (0 <= cnt <= lcap)
 *   list[ni][lcap]                the entries (0 <= entry < n, any order)
 * An entry equal to i is skipped: L_i of section 3.3 step 6 never holds i,
 * so a list that does gets no self-term.  Duplicated entries count twice.
 * Outputs
 *   acc[ni][3], jrk[ni][3]        F_I and dF_I
 *   sa[ni], sj[ni]                sums of m_j / r^2 and of
 *                                 m_j (|V| / r^3 + 3 |R.V| / r^4) over the
 *                                 same terms (may be NULL)
 *   pot[ni]                       irregular potential, -sum m_j / r over
 *                                 the list (may be NULL)
 * Returns 0, -1 for an index (idx or a list entry) outside [0, n), -3 for a
 * count outside [0, lcap]; nothing is computed then.
 */
int nb6o_irregular_force(int64_t n, const double *m, const double *xp,
                         const double *vp, int64_t ni, const int32_t *idx,
                         const int32_t *cnt, const int32_t *list, int64_t lcap,
                         double *acc, double *jrk, double *sa, double *sj,
                         double *pot, int nthreads)
{
    for (int64_t q = 0; q < ni; ++q) {
        if (idx[q] < 0 || idx[q] >= n) return -1;
        if (cnt[q] < 0 || cnt[q] > lcap) return -3;
        for (int64_t e = 0; e < cnt[q]; ++e)
            if (list[q * lcap + e] < 0 || list[q * lcap + e] >= n) return -1;
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif

#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < ni; ++q) {
        const int64_t i = idx[q];
        nsum A[3] = {{0, 0}, {0, 0}, {0, 0}};
        nsum J[3] = {{0, 0}, {0, 0}, {0, 0}};
        nsum SA = {0, 0}, SJ = {0, 0}, PHI = {0, 0};
        for (int64_t e = 0; e < cnt[q]; ++e) {
            const int64_t j = list[q * lcap + e];
            if (j == i) continue;
            const double mj = m[j];
            double Rij[3], Vij[3];
            for (int c = 0; c < 3; ++c) {
                Rij[c] = xp[3 * j + c] - xp[3 * i + c];
                Vij[c] = vp[3 * j + c] - vp[3 * i + c];
            }
            double d2 = Rij[0] * Rij[0] + Rij[1] * Rij[1] + Rij[2] * Rij[2];
            double d = sqrt(d2);
            double d3 = d2 * d;
            double d5 = d3 * d2;
            double rdotv = Rij[0] * Vij[0] + Rij[1] * Vij[1] + Rij[2] * Vij[2];
            for (int c = 0; c < 3; ++c) {
                nsum_add(&A[c], mj * Rij[c] / d3);
                nsum_add(&J[c], mj * (Vij[c] / d3 - 3.0 * rdotv * Rij[c] / d5));
            }
            double vabs = sqrt(Vij[0] * Vij[0] + Vij[1] * Vij[1] + Vij[2] * Vij[2]);
            nsum_add(&SA, mj / d2);
            nsum_add(&SJ, mj * (vabs / d3 + 3.0 * fabs(rdotv) / (d2 * d2)));
            nsum_add(&PHI, -mj / d);
        }
        for (int c = 0; c < 3; ++c) {
            acc[3 * q + c] = nsum_get(&A[c]);
            jrk[3 * q + c] = nsum_get(&J[c]);
        }
        if (sa) sa[q] = nsum_get(&SA);
        if (sj) sj[q] = nsum_get(&SJ);
        if (pot) pot[q] = nsum_get(&PHI);
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Regular corrector of a block (section 3.3 step 7, section 3.6, eq. 1)    */
/* ---------------------------------------------------------------------- */
/*
 * For each particle q of a block that reached its regular time t:
 *   h = t - t_old[q] (> 0), the length of its last regular step;
 *   the regular force change over the step with the neighbour set held
 *   fixed, section 3.6: the raw change plus the change of the irregular force
 *   at t from the old to the new list,
 *     dF  = (F_new - F_old)   + (G_new - G_old)
 *     dFd = (Fd_new - Fd_old) + (Gd_new - Gd_old)
 *   (F, Fd: regular force and derivative, at t_old for "old" and at t for
 *   "new"; G, Gd: irregular force and derivative at t with the old and the
 *   new list);
 *   the cubic through (F_old, Fd_old) at t_old and (F_old + dF, Fd_old + dFd)
 *   at t -- the fourth-order Hermite scheme (Makino & Aarseth 1992, which
 *   section 2 cites for the neighbour-change corrections) -- gives
 *     F2(t_old) = (6 dF - h (6 Fd_old + 2 dFd)) / h^2
 *     F3        = (-12 dF + 6 h (2 Fd_old + dFd)) / h^3
 *     F2(t)     = F2(t_old) + h F3;
 *   the next regular step: the standard criterion on the regular force at t,
 *     dt_est = sqrt(eta (|F_new| |F2(t)| + |Fd_new|^2)
 *                       / (|Fd_new| |F3| + |F2(t)|^2)),
 *   taken down to the largest power of two that is <= min(dt_est, 2 h,
 *   dt_max) and divides t (block steps stay commensurate with the block
 *   time, section 3.3 step 2), and not below dt_min;
 *   the new neighbour radius, equation (1):
 *     h_new = h_old f,  f = (n_p / n_nb)^(1/3) limited to [f_lo, f_hi],
 *     f = f_hi when the new list is empty (section 2: the empty case is
 *     catered for; the limits stand for its boundary modifications).
 * Arrays: t_old, h_old, n_p, dt_new, h_new [n]; nnb [n]; all vectors [n][3].
 * dt_min, dt_max: powers of two, dt_min <= dt_max; 0 < f_lo <= f_hi.
 * Returns 0, -1 for a bad parameter, -4 when some h <= 0 (nothing computed).
 */
static double pow2_floor_dividing(double limit, double t, double dt_min, double dt_max)
{
    double d = dt_max;
    while (d > dt_min && (d > limit || fmod(t, d) != 0.0)) d *= 0.5;
    return d;
}

static double norm3(const double *x)
{
    return sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
}

int nb6o_regular_correct(int64_t n, double t, const double *t_old,
                         const double *f_old, const double *fd_old,
                         const double *f_new, const double *fd_new,
                         const double *g_old, const double *gd_old,
                         const double *g_new, const double *gd_new,
                         const double *h_old, const int32_t *nnb, const double *n_p,
                         double eta, double dt_min, double dt_max, double f_lo,
                         double f_hi, double *df, double *dfd, double *f2,
                         double *f3, double *dt_new, double *h_new)
{
    int e_min, e_max;
    if (!(eta > 0.0) || !(dt_min > 0.0) || !(dt_max >= dt_min) ||
        frexp(dt_min, &e_min) != 0.5 || frexp(dt_max, &e_max) != 0.5 ||
        !(f_lo > 0.0) || !(f_hi >= f_lo))
        return -1;
    for (int64_t q = 0; q < n; ++q)
        if (!(t - t_old[q] > 0.0)) return -4;
    for (int64_t q = 0; q < n; ++q) {
        const double h = t - t_old[q];
        double F2[3], F3[3];
        for (int c = 0; c < 3; ++c) {
            const int64_t k = 3 * q + c;
            const double dF = (f_new[k] - f_old[k]) + (g_new[k] - g_old[k]);
            const double dFd = (fd_new[k] - fd_old[k]) + (gd_new[k] - gd_old[k]);
            const double f2_old = (6.0 * dF - h * (6.0 * fd_old[k] + 2.0 * dFd)) / (h * h);
            F3[c] = (-12.0 * dF + 6.0 * h * (2.0 * fd_old[k] + dFd)) / (h * h * h);
            F2[c] = f2_old + h * F3[c];
            df[k] = dF;
            dfd[k] = dFd;
            f2[k] = F2[c];
            f3[k] = F3[c];
        }
        const double a = norm3(f_new + 3 * q), ad = norm3(fd_new + 3 * q);
        const double a2 = norm3(F2), a3 = norm3(F3);
        const double est = sqrt(eta * (a * a2 + ad * ad) / (ad * a3 + a2 * a2));
        const double lim = fmin(fmin(est, 2.0 * h), dt_max);
        dt_new[q] = pow2_floor_dividing(lim, t, dt_min, dt_max);
        double f = f_hi;
        if (nnb[q] > 0) f = fmin(fmax(cbrt(n_p[q] / (double)nnb[q]), f_lo), f_hi);
        h_new[q] = h_old[q] * f;
    }
    return 0;
}

/* Number of OpenMP threads a parallel region of this library will use. */
int nb6o_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
