/*
 * Plain FP64 CPU oracle for the direct-sum n-body hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no source,
 * header, table or helper with the HIP library, and the HIP library never
 * loads it.
 *
 * What it computes, and where it comes from in the paper (Duy, Yamazaki,
 * Ikegami, Oyanagi, "Hybrid MPI-OpenMP Paradigm on SMP clusters: MPEG-2
 * Encoder and n-body Simulation"):
 *
 *   oracle_accel     Section IV (problem statement) and Section IV.A (the
 *                    force loop over an interaction list): with every cell of
 *                    the tree opened, the interaction list of body i is every
 *                    other body, and the force is the exact pairwise sum.
 *                    Plummer softening eps, gravitational constant G.
 *                      a_i   =  G sum_{j != i} m_j (x_j - x_i) / (r_ij^2 + eps^2)^(3/2)
 *                      phi_i = -G sum_{j != i} m_j / (r_ij^2 + eps^2)^(1/2)
 *                    Sums run over j = 0..n-1 in index order, skipping j = i,
 *                    with Neumaier-compensated FP64 accumulation.
 *   oracle_leapfrog  Section IV.A, last step, and the pseudo-code of Section
 *                    IV.B (Move_bodies after the force calculation): bodies
 *                    update velocity and position from the computed forces.
 *                    The integrator is read as kick-drift-kick leapfrog with
 *                    one force evaluation per step.
 *   oracle_energy    Diagnostics of that integration: K = 1/2 sum m |v|^2,
 *                    U = 1/2 sum m phi.
 *   oracle_orb_order Section IV.B, Orthogonal Recursive Bisection: split the
 *                    body set into non-overlapping sub-spaces holding about
 *                    equal numbers of bodies, recursively, here down to
 *                    leaves of at most `leaf` bodies.  The exact splitting
 *                    rule (longest FP32 extent, IEEE total order plus index
 *                    as the key, leaf-aligned left count, leaves sorted by
 *                    index) is this library's reading of that sentence.
 *   oracle_vjp       Reverse-mode derivative (vector-Jacobian product) of
 *                    oracle_accel with respect to positions and masses,
 *                    written from the derivative of the pair law (the paper
 *                    has no derivatives).
 *   oracle_traj_grad Reverse mode through oracle_leapfrog for the loss
 *                    L = sum_i |x_i(T) - y_i|^2, storing every state;
 *                    oracle_traj_grad_cot takes any cotangents of the final
 *                    state, including one of the final potential.
 *   oracle_janus_run Bit-reversible fixed-point form of the same
 *                    kick-drift-kick (integer state, increments rounded once),
 *                    forward or backward.
 *   oracle_tree_*    Section IV.A tree code (cells replaced by their total
 *                    mass at their centre of mass when distant enough, found
 *                    by a walk from the root) on the cells of the Section
 *                    IV.B ORB recursion: node table, moments, interaction
 *                    lists and the resulting force; the readings are stated
 *                    above those functions.
 *   oracle_tree_pseudo, oracle_tree_quad, oracle_tree_accel_cells
 *                    Higher-order cells, after the pseudo-particle multipole
 *                    method of Makino (J. Comput. Phys. 151, 1999), the
 *                    paper's reference [20], which Section VI cites for
 *                    the O(N) fast multipole method:
 *                    each cell's expansion to quadrupole order is carried
 *                    either by 12 point masses from that method's formula,
 *                    or by the cell's traceless quadrupole tensor with the
 *                    expansion evaluated directly; and the fast multipole
 *                    method's local expansions at the level of the target
 *                    groups (cells far from a whole group enter one Taylor
 *                    expansion about the group's centre).
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (no fast-math;
 * contraction off so that every product and sum rounds as written).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Neumaier's improvement of Kahan summation: exact running error term. */
typedef struct { double s, c; } nsum;

static inline void nsum_add(nsum *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v))
        a->c += (a->s - t) + v;
    else
        a->c += (v - t) + a->s;
    a->s = t;
}

static inline double nsum_val(const nsum *a) { return a->s + a->c; }

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------------------
 * Force and potential by direct summation.
 * x: [n][3] positions, m: [n] masses.  targets: NULL for all n bodies (then
 * ntarg must equal n), else ntarg indices in [0, n).  acc: [ntarg][3],
 * pot: [ntarg] (either may be NULL).
 * ------------------------------------------------------------------------- */
void oracle_accel(int64_t n, const double *x, const double *m, double G, double eps,
                  int64_t ntarg, const int64_t *targets, double *acc, double *pot)
{
    const double eps2 = eps * eps;
    int64_t t;
#pragma omp parallel for schedule(dynamic, 64)
    for (t = 0; t < ntarg; ++t) {
        const int64_t i = targets ? targets[t] : t;
        const double xi = x[3 * i], yi = x[3 * i + 1], zi = x[3 * i + 2];
        nsum ax = {0, 0}, ay = {0, 0}, az = {0, 0}, ph = {0, 0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i)
                continue;
            const double dx = x[3 * j] - xi;
            const double dy = x[3 * j + 1] - yi;
            const double dz = x[3 * j + 2] - zi;
            const double r2 = ((dx * dx + dy * dy) + dz * dz) + eps2;
            const double r = sqrt(r2);
            const double w = 1.0 / (r2 * r); /* (r^2 + eps^2)^(-3/2) */
            const double mw = m[j] * w;
            nsum_add(&ax, mw * dx);
            nsum_add(&ay, mw * dy);
            nsum_add(&az, mw * dz);
            nsum_add(&ph, m[j] / r);
        }
        if (acc) {
            acc[3 * t] = G * nsum_val(&ax);
            acc[3 * t + 1] = G * nsum_val(&ay);
            acc[3 * t + 2] = G * nsum_val(&az);
        }
        if (pot)
            pot[t] = -G * nsum_val(&ph);
    }
}

/* ---------------------------------------------------------------------------
 * Energies: out[0] = K = 1/2 sum m |v|^2, out[1] = U = 1/2 sum m phi.
 * v: [n][3].
 * ------------------------------------------------------------------------- */
void oracle_energy(int64_t n, const double *v, const double *m, const double *pot, double *out)
{
    nsum k = {0, 0}, u = {0, 0};
    for (int64_t i = 0; i < n; ++i) {
        const double v2 = (v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1]) + v[3 * i + 2] * v[3 * i + 2];
        nsum_add(&k, 0.5 * m[i] * v2);
        nsum_add(&u, 0.5 * m[i] * pot[i]);
    }
    out[0] = nsum_val(&k);
    out[1] = nsum_val(&u);
}

/* ---------------------------------------------------------------------------
 * Kick-drift-kick leapfrog, one force evaluation per step, h = dt/2:
 *   v <- v + h a(x);  x <- x + dt v;  a <- a(x);  v <- v + h a.
 * x, v: [n][3] in/out.  acc [n][3], pot [n]: out (the force at the final
 * positions).  The force at the initial positions is evaluated first.
 * energy: NULL or [(nsteps+1)][2] = (K, U) after each step, entry 0 at t=0.
 * ------------------------------------------------------------------------- */
void oracle_leapfrog(int64_t n, double *x, double *v, const double *m, double G, double eps,
                     double dt, int32_t nsteps, double *acc, double *pot, double *energy)
{
    const double h = 0.5 * dt;
    oracle_accel(n, x, m, G, eps, n, NULL, acc, pot);
    if (energy)
        oracle_energy(n, v, m, pot, energy);
    for (int32_t s = 0; s < nsteps; ++s) {
        for (int64_t k = 0; k < 3 * n; ++k)
            v[k] = v[k] + h * acc[k];
        for (int64_t k = 0; k < 3 * n; ++k)
            x[k] = x[k] + dt * v[k];
        oracle_accel(n, x, m, G, eps, n, NULL, acc, pot);
        for (int64_t k = 0; k < 3 * n; ++k)
            v[k] = v[k] + h * acc[k];
        if (energy)
            oracle_energy(n, v, m, pot, energy + 2 * (s + 1));
    }
}

/* ---------------------------------------------------------------------------
 * Orthogonal Recursive Bisection order.
 * xf: [n][3] FP32 coordinates.  perm: [n] out, perm[p] = original index of
 * the body placed at position p.  Returns 0, or -1 on bad arguments.
 *
 * ORB(S):
 *   |S| <= leaf: emit S by ascending original index.
 *   else: FP32 bounding box of S; extent_k = fl32(max_k - min_k); axis = the
 *   largest extent, ties to the lowest axis (x, then y, then z).  Key of body
 *   i = (T(coord_axis(i)), i), compared lexicographically, where T maps the
 *   FP32 bit pattern to its IEEE total order as an unsigned integer.  With
 *   L = ceil(|S| / leaf), the left part is the k = leaf * ceil(L / 2)
 *   smallest keys, the right part the rest; emit ORB(left) then ORB(right).
 * ------------------------------------------------------------------------- */
static uint32_t total_order_bits(float f)
{
    uint32_t u;
    memcpy(&u, &f, sizeof u);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

typedef struct { uint64_t key; int32_t idx; } orb_item;

static int cmp_item(const void *a, const void *b)
{
    const orb_item *p = (const orb_item *)a, *q = (const orb_item *)b;
    return (p->key > q->key) - (p->key < q->key);
}

static int cmp_i32(const void *a, const void *b)
{
    const int32_t p = *(const int32_t *)a, q = *(const int32_t *)b;
    return (p > q) - (p < q);
}

static void orb_rec(const float *xf, int32_t *s, int64_t cnt, int32_t leaf, orb_item *tmp)
{
    if (cnt <= leaf) {
        qsort(s, (size_t)cnt, sizeof(int32_t), cmp_i32);
        return;
    }
    float lo[3], hi[3];
    for (int k = 0; k < 3; ++k)
        lo[k] = hi[k] = xf[3 * (int64_t)s[0] + k];
    for (int64_t p = 1; p < cnt; ++p)
        for (int k = 0; k < 3; ++k) {
            const float c = xf[3 * (int64_t)s[p] + k];
            if (c < lo[k])
                lo[k] = c;
            if (c > hi[k])
                hi[k] = c;
        }
    float ext[3];
    for (int k = 0; k < 3; ++k)
        ext[k] = hi[k] - lo[k]; /* one FP32 subtraction, rounded to nearest */
    int axis = 0;
    if (ext[1] > ext[axis])
        axis = 1;
    if (ext[2] > ext[axis])
        axis = 2;
    for (int64_t p = 0; p < cnt; ++p) {
        tmp[p].idx = s[p];
        tmp[p].key = ((uint64_t)total_order_bits(xf[3 * (int64_t)s[p] + axis]) << 32) | (uint32_t)s[p];
    }
    qsort(tmp, (size_t)cnt, sizeof(orb_item), cmp_item);
    for (int64_t p = 0; p < cnt; ++p)
        s[p] = tmp[p].idx;
    const int64_t L = (cnt + leaf - 1) / leaf;
    int64_t k = (int64_t)leaf * ((L + 1) / 2);
    if (k > cnt)
        k = cnt;
    orb_rec(xf, s, k, leaf, tmp);
    orb_rec(xf, s + k, cnt - k, leaf, tmp);
}

int oracle_orb_order(int64_t n, const float *xf, int32_t leaf, int32_t *perm)
{
    if (n < 1 || n > 0x7fffffff || leaf < 1 || !xf || !perm)
        return -1;
    for (int64_t i = 0; i < n; ++i)
        perm[i] = (int32_t)i;
    orb_item *tmp = (orb_item *)malloc((size_t)n * sizeof(orb_item));
    if (!tmp)
        return -1;
    orb_rec(xf, perm, n, leaf, tmp);
    free(tmp);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Vector-Jacobian product of (a, phi) with respect to (x, m).
 * With d = x_j - x_k, q = r^2 + eps^2, w = q^(-3/2), u = q^(-5/2) and
 * T_kj = w I - 3 u d d^T (symmetric, T_kj = T_jk):
 *   da_i/dx_j = G m_j T_ij (j != i),  da_i/dx_i = -G sum_j m_j T_ij,
 *   da_i/dm_j = G w_ij (x_j - x_i),
 *   dphi_i/dx_j = G m_j w_ij (x_j - x_i),  dphi_i/dx_i = -a_i,
 *   dphi_i/dm_j = -G q_ij^(-1/2).
 * Hence, for cotangents abar (on a) and phibar (on phi):
 *   xbar_k = G sum_{j!=k} T_kj (m_k abar_j - m_j abar_k)
 *            - G m_k sum_{j!=k} phibar_j w_kj d_kj  - phibar_k a_k
 *   mbar_k = -G sum_{j!=k} w_kj d_kj . abar_j  - G sum_{j!=k} phibar_j q_kj^(-1/2)
 * x: [n][3], abar: [n][3], phibar: [n] or NULL, xbar: [n][3], mbar: [n].
 * ------------------------------------------------------------------------- */
void oracle_vjp(int64_t n, const double *x, const double *m, double G, double eps,
                const double *abar, const double *phibar, double *xbar, double *mbar)
{
    const double eps2 = eps * eps;
    int64_t k;
#pragma omp parallel for schedule(dynamic, 64)
    for (k = 0; k < n; ++k) {
        const double xk = x[3 * k], yk = x[3 * k + 1], zk = x[3 * k + 2];
        const double ak0 = abar[3 * k], ak1 = abar[3 * k + 1], ak2 = abar[3 * k + 2];
        nsum gx = {0, 0}, gy = {0, 0}, gz = {0, 0}, gm = {0, 0};
        nsum fx = {0, 0}, fy = {0, 0}, fz = {0, 0}; /* a_k / G, for the phibar term */
        for (int64_t j = 0; j < n; ++j) {
            if (j == k)
                continue;
            const double d0 = x[3 * j] - xk, d1 = x[3 * j + 1] - yk, d2 = x[3 * j + 2] - zk;
            const double q = ((d0 * d0 + d1 * d1) + d2 * d2) + eps2;
            const double r = sqrt(q);
            const double w = 1.0 / (q * r);
            const double u = w / q;
            /* e = m_k abar_j - m_j abar_k */
            const double e0 = m[k] * abar[3 * j] - m[j] * ak0;
            const double e1 = m[k] * abar[3 * j + 1] - m[j] * ak1;
            const double e2 = m[k] * abar[3 * j + 2] - m[j] * ak2;
            const double de = (d0 * e0 + d1 * e1) + d2 * e2;
            /* T e = w e - 3 u d (d . e) */
            nsum_add(&gx, w * e0 - 3.0 * u * d0 * de);
            nsum_add(&gy, w * e1 - 3.0 * u * d1 * de);
            nsum_add(&gz, w * e2 - 3.0 * u * d2 * de);
            const double da = (d0 * abar[3 * j] + d1 * abar[3 * j + 1]) + d2 * abar[3 * j + 2];
            nsum_add(&gm, -w * da);
            if (phibar) {
                nsum_add(&gx, -m[k] * phibar[j] * w * d0);
                nsum_add(&gy, -m[k] * phibar[j] * w * d1);
                nsum_add(&gz, -m[k] * phibar[j] * w * d2);
                nsum_add(&gm, -phibar[j] / r);
                nsum_add(&fx, m[j] * w * d0);
                nsum_add(&fy, m[j] * w * d1);
                nsum_add(&fz, m[j] * w * d2);
            }
        }
        xbar[3 * k] = G * nsum_val(&gx);
        xbar[3 * k + 1] = G * nsum_val(&gy);
        xbar[3 * k + 2] = G * nsum_val(&gz);
        mbar[k] = G * nsum_val(&gm);
        if (phibar) {
            xbar[3 * k] -= phibar[k] * G * nsum_val(&fx);
            xbar[3 * k + 1] -= phibar[k] * G * nsum_val(&fy);
            xbar[3 * k + 2] -= phibar[k] * G * nsum_val(&fz);
        }
    }
}

/* ---------------------------------------------------------------------------
 * Gradient of L = sum_i |x_i(T) - y_i|^2 through nsteps of the leapfrog
 * above, with respect to x0, v0 and m.  Plain reverse mode: the forward pass
 * stores every position x_0..x_T; the reverse pass visits the operations in
 * the opposite order (closing kick, force, drift, opening kick) and ends with
 * the force at x_0.  Returns L.  y, gx, gv: [n][3]; gm: [n].
 * ------------------------------------------------------------------------- */
/* ---------------------------------------------------------------------------
 * Reverse mode through oracle_leapfrog for given cotangents of the final
 * state: xbar_T, vbar_T ([n][3]) and phibar_T ([n], the cotangent of the
 * potential phi(x_T), may be NULL).  Returns dL/dx0, dL/dv0, dL/dm through
 * the trajectory (the explicit dependence of the loss on m is the caller's).
 * The phibar path: phi(x_T) is one more evaluation of the pair law at x_T, so
 * its cotangent enters through one VJP with abar = 0 before the reverse loop.
 * ------------------------------------------------------------------------- */
int oracle_traj_grad_cot(int64_t n, const double *x0, const double *v0, const double *m, double G,
                         double eps, double dt, int32_t nsteps, const double *xbar_T,
                         const double *vbar_T, const double *phibar_T, double *gx, double *gv,
                         double *gm)
{
    const double h = 0.5 * dt;
    const size_t n3 = (size_t)(3 * n);
    double *xs = (double *)malloc((size_t)(nsteps + 1) * n3 * sizeof(double));
    double *v = (double *)malloc(n3 * sizeof(double));
    double *a = (double *)malloc(n3 * sizeof(double));
    double *abar = (double *)malloc(n3 * sizeof(double));
    double *tx = (double *)malloc(n3 * sizeof(double));
    double *tm = (double *)malloc((size_t)n * sizeof(double));
    if (!xs || !v || !a || !abar || !tx || !tm) {
        free(xs); free(v); free(a); free(abar); free(tx); free(tm);
        return -1;
    }
    memcpy(xs, x0, n3 * sizeof(double));
    memcpy(v, v0, n3 * sizeof(double));
    oracle_accel(n, xs, m, G, eps, n, NULL, a, NULL);
    for (int32_t s = 0; s < nsteps; ++s) {
        const double *xc = xs + (size_t)s * n3;
        double *xn = xs + (size_t)(s + 1) * n3;
        for (size_t k = 0; k < n3; ++k)
            v[k] = v[k] + h * a[k];
        for (size_t k = 0; k < n3; ++k)
            xn[k] = xc[k] + dt * v[k];
        oracle_accel(n, xn, m, G, eps, n, NULL, a, NULL);
        for (size_t k = 0; k < n3; ++k)
            v[k] = v[k] + h * a[k];
    }
    for (size_t k = 0; k < n3; ++k) {
        gx[k] = xbar_T[k];
        gv[k] = vbar_T[k];
    }
    for (int64_t k = 0; k < n; ++k)
        gm[k] = 0.0;
    if (phibar_T) {
        for (size_t k = 0; k < n3; ++k)
            abar[k] = 0.0;
        oracle_vjp(n, xs + (size_t)nsteps * n3, m, G, eps, abar, phibar_T, tx, tm);
        for (size_t k = 0; k < n3; ++k)
            gx[k] += tx[k];
        for (int64_t k = 0; k < n; ++k)
            gm[k] += tm[k];
    }
    double *carry = a;
    for (size_t k = 0; k < n3; ++k)
        carry[k] = 0.0;
    for (int32_t s = nsteps - 1; s >= 0; --s) {
        const double *xn = xs + (size_t)(s + 1) * n3;
        for (size_t k = 0; k < n3; ++k)
            abar[k] = h * gv[k] + carry[k];
        oracle_vjp(n, xn, m, G, eps, abar, NULL, tx, tm);
        for (size_t k = 0; k < n3; ++k)
            gx[k] += tx[k];
        for (int64_t k = 0; k < n; ++k)
            gm[k] += tm[k];
        for (size_t k = 0; k < n3; ++k)
            gv[k] += dt * gx[k];
        for (size_t k = 0; k < n3; ++k)
            carry[k] = h * gv[k];
    }
    oracle_vjp(n, xs, m, G, eps, carry, NULL, tx, tm);
    for (size_t k = 0; k < n3; ++k)
        gx[k] += tx[k];
    for (int64_t k = 0; k < n; ++k)
        gm[k] += tm[k];
    free(xs); free(v); free(a); free(abar); free(tx); free(tm);
    return 0;
}

double oracle_traj_grad(int64_t n, const double *x0, const double *v0, const double *m,
                        const double *y, double G, double eps, double dt, int32_t nsteps,
                        double *gx, double *gv, double *gm)
{
    const double h = 0.5 * dt;
    const size_t n3 = (size_t)(3 * n);
    double *xs = (double *)malloc((size_t)(nsteps + 1) * n3 * sizeof(double));
    double *v = (double *)malloc(n3 * sizeof(double));
    double *a = (double *)malloc(n3 * sizeof(double));
    double *abar = (double *)malloc(n3 * sizeof(double));
    double *tx = (double *)malloc(n3 * sizeof(double));
    double *tm = (double *)malloc((size_t)n * sizeof(double));
    if (!xs || !v || !a || !abar || !tx || !tm) {
        free(xs); free(v); free(a); free(abar); free(tx); free(tm);
        return NAN;
    }
    /* forward */
    memcpy(xs, x0, n3 * sizeof(double));
    memcpy(v, v0, n3 * sizeof(double));
    oracle_accel(n, xs, m, G, eps, n, NULL, a, NULL);
    for (int32_t s = 0; s < nsteps; ++s) {
        const double *xc = xs + (size_t)s * n3;
        double *xn = xs + (size_t)(s + 1) * n3;
        for (size_t k = 0; k < n3; ++k)
            v[k] = v[k] + h * a[k];
        for (size_t k = 0; k < n3; ++k)
            xn[k] = xc[k] + dt * v[k];
        oracle_accel(n, xn, m, G, eps, n, NULL, a, NULL);
        for (size_t k = 0; k < n3; ++k)
            v[k] = v[k] + h * a[k];
    }
    const double *xT = xs + (size_t)nsteps * n3;
    nsum L = {0, 0};
    for (size_t k = 0; k < n3; ++k) {
        const double d = xT[k] - y[k];
        nsum_add(&L, d * d);
        gx[k] = 2.0 * d; /* xbar_T */
        gv[k] = 0.0;     /* vbar_T */
    }
    for (int64_t k = 0; k < n; ++k)
        gm[k] = 0.0;
    /* reverse; carry = cotangent on a(x_{s+1}) from the opening kick of
     * step s+1, which the later iteration has already visited */
    double *carry = a;
    for (size_t k = 0; k < n3; ++k)
        carry[k] = 0.0;
    for (int32_t s = nsteps - 1; s >= 0; --s) {
        const double *xn = xs + (size_t)(s + 1) * n3;
        /* closing kick v_{s+1} = v_half + h a(x_{s+1}) */
        for (size_t k = 0; k < n3; ++k)
            abar[k] = h * gv[k] + carry[k];
        /* force a(x_{s+1}) */
        oracle_vjp(n, xn, m, G, eps, abar, NULL, tx, tm);
        for (size_t k = 0; k < n3; ++k)
            gx[k] += tx[k];
        for (int64_t k = 0; k < n; ++k)
            gm[k] += tm[k];
        /* drift x_{s+1} = x_s + dt v_half */
        for (size_t k = 0; k < n3; ++k)
            gv[k] += dt * gx[k];
        /* opening kick v_half = v_s + h a(x_s) */
        for (size_t k = 0; k < n3; ++k)
            carry[k] = h * gv[k];
    }
    /* the force at x_0, used by the opening kick of step 0 */
    oracle_vjp(n, xs, m, G, eps, carry, NULL, tx, tm);
    for (size_t k = 0; k < n3; ++k)
        gx[k] += tx[k];
    for (int64_t k = 0; k < n; ++k)
        gm[k] += tm[k];
    const double out = nsum_val(&L);
    free(xs); free(v); free(a); free(abar); free(tx); free(tm);
    return out;
}

/* ---------------------------------------------------------------------------
 * Tree code on the ORB hierarchy.
 *
 * Section IV.A: a distant group of bodies is replaced by one body of the
 * group's total mass at its centre of mass; the force on a body is found by
 * walking the tree from the root, adding a cell to the interaction list when
 * it is distant enough and otherwise visiting its children, then summing over
 * the list of cells and bodies.  Section IV.B: the space is divided by ORB.
 * Here the cells are the nodes of the ORB recursion itself (the readings
 * below are this library's, the paper fixes none of them):
 *
 *   nodes     node k covers ORB positions [begin, end); a node of more than
 *             `leaf` bodies splits at begin + leaf*ceil(L/2), L =
 *             ceil(size/leaf), exactly as in oracle_orb_order.  Nodes are
 *             numbered in preorder (node, left subtree, right subtree).
 *   groups    the targets are taken in groups: the maximal nodes of at
 *             most `group` bodies (group >= leaf), in ORB order.  One walk
 *             serves every body of a group.
 *   moments   in FP64 from the FP32 inputs: a leaf sums m and m*x over its
 *             positions in order starting from 0 (product rounded, then
 *             added); an inner node adds left + right.  com = (sum m x) / M,
 *             or the box centre 0.5*(lo + hi) when M = 0.  The box lo/hi is
 *             the exact coordinate minimum/maximum; diag2 = sum over axes of
 *             (hi - lo)^2, axes in order x, y, z.
 *   opening   cell c is accepted for group g iff c and g share no body
 *             (neither contains the other) and
 *             diag2_c < theta^2 * D2, where D2 is the squared distance from
 *             com_c to the box of g (per axis lo - com if com < lo, com - hi
 *             if com > hi, else 0; summed x, y, z).  Every body of g is then
 *             at least D = sqrt(D2) from com_c while every body of c lies
 *             within sqrt(diag2_c) of it, so the ratio of cell size to
 *             distance is below theta for each body of the group.
 *   walk      visit(c): accept -> far list; else a leaf -> near list; else
 *             visit(left), visit(right).  Starts at the root.
 *   force     far cells act as a body of mass M at com (same softened law);
 *             near leaves act body by body, skipping the target itself.
 * theta = 0 never accepts a cell, so the tree force is the direct sum.
 * Masses must be non-negative.
 * ------------------------------------------------------------------------- */
static int64_t tree_count_rec(int64_t size, int32_t leaf)
{
    if (size <= leaf)
        return 1;
    const int64_t L = (size + leaf - 1) / leaf;
    int64_t k = (int64_t)leaf * ((L + 1) / 2);
    if (k > size)
        k = size;
    return 1 + tree_count_rec(k, leaf) + tree_count_rec(size - k, leaf);
}

static int64_t tree_build_rec(int64_t b, int64_t size, int32_t leaf, int64_t *nodes, int64_t *next)
{
    const int64_t id = (*next)++;
    nodes[4 * id] = b;
    nodes[4 * id + 1] = b + size;
    if (size <= leaf) {
        nodes[4 * id + 2] = -1;
        nodes[4 * id + 3] = -1;
        return id;
    }
    const int64_t L = (size + leaf - 1) / leaf;
    int64_t k = (int64_t)leaf * ((L + 1) / 2);
    if (k > size)
        k = size;
    const int64_t l = tree_build_rec(b, k, leaf, nodes, next);
    const int64_t r = tree_build_rec(b + k, size - k, leaf, nodes, next);
    nodes[4 * id + 2] = l;
    nodes[4 * id + 3] = r;
    return id;
}

/* Returns the node count; fills nodes[nn][4] = (begin, end, left, right) when
 * nodes is not NULL (left = right = -1 for a leaf). */
int64_t oracle_tree_nodes(int64_t n, int32_t leaf, int64_t *nodes)
{
    if (n < 1 || leaf < 1)
        return -1;
    const int64_t nn = tree_count_rec(n, leaf);
    if (nodes) {
        int64_t next = 0;
        tree_build_rec(0, n, leaf, nodes, &next);
    }
    return nn;
}

/* Moments of every node.  x: [n][3], m: [n] in ORB order (FP32 values widened
 * to FP64).  mass: [nn], com: [nn][3], lo/hi: [nn][3], diag2: [nn]. */
static void tree_moments_rec(const int64_t *nodes, int64_t id, const double *x, const double *m,
                             double *mass, double *sx, double *lo, double *hi)
{
    const int64_t b = nodes[4 * id], e = nodes[4 * id + 1];
    const int64_t l = nodes[4 * id + 2], r = nodes[4 * id + 3];
    if (l < 0) {
        double M = 0.0, s[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < 3; ++k)
            lo[3 * id + k] = hi[3 * id + k] = x[3 * b + k];
        for (int64_t p = b; p < e; ++p) {
            M = M + m[p];
            for (int k = 0; k < 3; ++k) {
                const double c = x[3 * p + k];
                const double mc = m[p] * c;
                s[k] = s[k] + mc;
                if (c < lo[3 * id + k])
                    lo[3 * id + k] = c;
                if (c > hi[3 * id + k])
                    hi[3 * id + k] = c;
            }
        }
        mass[id] = M;
        for (int k = 0; k < 3; ++k)
            sx[3 * id + k] = s[k];
        return;
    }
    tree_moments_rec(nodes, l, x, m, mass, sx, lo, hi);
    tree_moments_rec(nodes, r, x, m, mass, sx, lo, hi);
    mass[id] = mass[l] + mass[r];
    for (int k = 0; k < 3; ++k) {
        sx[3 * id + k] = sx[3 * l + k] + sx[3 * r + k];
        lo[3 * id + k] = lo[3 * l + k] < lo[3 * r + k] ? lo[3 * l + k] : lo[3 * r + k];
        hi[3 * id + k] = hi[3 * l + k] > hi[3 * r + k] ? hi[3 * l + k] : hi[3 * r + k];
    }
}

int oracle_tree_moments(int64_t n, int32_t leaf, const double *x, const double *m, double *mass,
                        double *com, double *lo, double *hi, double *diag2)
{
    const int64_t nn = oracle_tree_nodes(n, leaf, NULL);
    if (nn < 1)
        return -1;
    int64_t *nodes = (int64_t *)malloc((size_t)nn * 4 * sizeof(int64_t));
    double *sx = (double *)malloc((size_t)nn * 3 * sizeof(double));
    if (!nodes || !sx) {
        free(nodes);
        free(sx);
        return -1;
    }
    oracle_tree_nodes(n, leaf, nodes);
    tree_moments_rec(nodes, 0, x, m, mass, sx, lo, hi);
    for (int64_t id = 0; id < nn; ++id) {
        for (int k = 0; k < 3; ++k) {
            if (mass[id] > 0.0)
                com[3 * id + k] = sx[3 * id + k] / mass[id];
            else
                com[3 * id + k] = 0.5 * (lo[3 * id + k] + hi[3 * id + k]);
        }
        double d2 = 0.0;
        for (int k = 0; k < 3; ++k) {
            const double ext = hi[3 * id + k] - lo[3 * id + k];
            d2 = d2 + ext * ext;
        }
        diag2[id] = d2;
    }
    free(nodes);
    free(sx);
    return 0;
}

typedef struct {
    const int64_t *nodes;
    const double *com, *lo, *hi, *diag2;
    double theta2;
} tree_ctx;

static int tree_accept(const tree_ctx *t, int64_t c, int64_t g)
{
    const int64_t *nc = t->nodes + 4 * c, *ng = t->nodes + 4 * g;
    if (nc[0] < ng[1] && ng[0] < nc[1])
        return 0; /* c and the group overlap: c contains it or lies inside it */
    double d[3];
    for (int k = 0; k < 3; ++k) {
        const double p = t->com[3 * c + k];
        const double a = t->lo[3 * g + k], b = t->hi[3 * g + k];
        d[k] = p < a ? a - p : (p > b ? p - b : 0.0);
    }
    const double D2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    return t->diag2[c] < t->theta2 * D2;
}

/* Walk for group node g; appends to far/near (either may be NULL to count). */
static void tree_walk_rec(const tree_ctx *t, int64_t c, int64_t g, int32_t *far, int64_t *nf,
                          int32_t *near, int64_t *nnr)
{
    if (tree_accept(t, c, g)) {
        if (far)
            far[*nf] = (int32_t)c;
        ++*nf;
        return;
    }
    const int64_t l = t->nodes[4 * c + 2], r = t->nodes[4 * c + 3];
    if (l < 0) {
        if (near)
            near[*nnr] = (int32_t)c;
        ++*nnr;
        return;
    }
    tree_walk_rec(t, l, g, far, nf, near, nnr);
    tree_walk_rec(t, r, g, far, nf, near, nnr);
}

/* ---------------------------------------------------------------------------
 * Group local expansions (the M2L and L2P steps of the fast multipole method
 * the paper's Section VI points to through its reference [20], taken at the
 * level of the target groups; cells carry their quadrupole expansion).
 * Readings of this library:
 *   centre   z_g = the group node's FP64 centre of mass.
 *   MAC_L    cell c may enter group g's local expansion iff c and g share no
 *            body and diag2_c + diag2_g < theta^2 |com_c - z_g|^2.  Every
 *            body of c is within sqrt(diag2_c) of com_c and every target
 *            within sqrt(diag2_g) of z_g, and (b_c + b_g)^2 <= 2 (b_c^2 +
 *            b_g^2), so both expansions converge for theta < 1/sqrt(2)
 *            and their size-to-distance ratio is below sqrt(2) theta; no
 *            square roots.
 *   walk     visit(c): MAC_L -> local list; else the monopole acceptance
 *            test -> far list, evaluated body by body as a quadrupole cell;
 *            else a leaf -> near list; else visit(left), visit(right).  The
 *            far and near lists are thus never longer than those of the
 *            quadrupole cells alone.
 *   M2L      the cell's potential sum P_c(x) = M/s + (r.Q.r)/(2 s^5),
 *            r = x - com_c, s^2 = |r|^2 + eps^2, expanded to third order
 *            about z_g (one order above the cells', so that the force,
 *            which loses one order, keeps the cells' third-order error):
 *            P0 = P_c(z_g), p = grad P_c, K = grad grad P_c, T = the third
 *            derivatives, at z_g, with r = z_g - com_c and q = Q r:
 *              p_k   = -M r_k/s^3 - 5 (r.Q.r) r_k / (2 s^7) + q_k / s^5
 *              K_kl  = M (3 r_k r_l / s^5 - delta_kl / s^3)
 *                      + 35 (r.Q.r) r_k r_l / (2 s^9)
 *                      - 5 (2 q_k r_l + 2 q_l r_k + delta_kl r.Q.r) / (2 s^7)
 *                      + Q_kl / s^5
 *              T_klm = M (-15 r_k r_l r_m / s^7 + 3 (d_kl r_m + d_km r_l + d_lm r_k) / s^5)
 *                      - 315 (r.Q.r) r_k r_l r_m / (2 s^11)
 *                      + 35 (q_k r_l r_m + q_l r_k r_m + q_m r_k r_l) / s^9
 *                      + 35 (r.Q.r) (d_kl r_m + d_km r_l + d_lm r_k) / (2 s^9)
 *                      - 5 (Q_kl r_m + Q_km r_l + Q_lm r_k + q_k d_lm + q_l d_km + q_m d_kl) / s^7
 *            (d = Kronecker delta), summed over the local list in walk order
 *            (Neumaier).
 *   L2P      at y = x - z_g: a += G (p + K y + T(y, y) / 2),
 *            phi -= G (P0 + p.y + y.K.y / 2 + T(y, y, y) / 6).
 * ------------------------------------------------------------------------- */
static int tree_overlap(const int64_t *nodes, int64_t c, int64_t g)
{
    const int64_t *nc = nodes + 4 * c, *ng = nodes + 4 * g;
    return nc[0] < ng[1] && ng[0] < nc[1];
}

static double tree_centre_dist2(const tree_ctx *t, int64_t c, int64_t g)
{
    const double dx = t->com[3 * c] - t->com[3 * g];
    const double dy = t->com[3 * c + 1] - t->com[3 * g + 1];
    const double dz = t->com[3 * c + 2] - t->com[3 * g + 2];
    return (dx * dx + dy * dy) + dz * dz;
}

/* Local-expansion walk for group node g: appends to loc/far/near (any may be
 * NULL to count). */
static void tree_walk_local_rec(const tree_ctx *t, int64_t c, int64_t g, int32_t *loc, int64_t *nl, int32_t *far,
                                int64_t *nf, int32_t *near, int64_t *nnr)
{
    if (!tree_overlap(t->nodes, c, g)) {
        const double dz2 = tree_centre_dist2(t, c, g);
        if (t->diag2[c] + t->diag2[g] < t->theta2 * dz2) {
            if (loc)
                loc[*nl] = (int32_t)c;
            ++*nl;
            return;
        }
        if (tree_accept(t, c, g)) {
            if (far)
                far[*nf] = (int32_t)c;
            ++*nf;
            return;
        }
    }
    const int64_t l = t->nodes[4 * c + 2], r = t->nodes[4 * c + 3];
    if (l < 0) {
        if (near)
            near[*nnr] = (int32_t)c;
        ++*nnr;
        return;
    }
    tree_walk_local_rec(t, l, g, loc, nl, far, nf, near, nnr);
    tree_walk_local_rec(t, r, g, loc, nl, far, nf, near, nnr);
}

typedef struct {
    int64_t nn, ngroups;
    int64_t *nodes, *group_node;
    double *mass, *com, *lo, *hi, *diag2;
} tree_data;

/* Collects the groups under node id in preorder. */
static void tree_groups_rec(const int64_t *nodes, int64_t id, int64_t group, int64_t *out, int64_t *cnt)
{
    const int64_t size = nodes[4 * id + 1] - nodes[4 * id];
    if (size <= group || nodes[4 * id + 2] < 0) {
        if (out)
            out[*cnt] = id;
        ++*cnt;
        return;
    }
    tree_groups_rec(nodes, nodes[4 * id + 2], group, out, cnt);
    tree_groups_rec(nodes, nodes[4 * id + 3], group, out, cnt);
}

static void tree_free(tree_data *d)
{
    free(d->nodes);
    free(d->group_node);
    free(d->mass);
    free(d->com);
    free(d->lo);
    free(d->hi);
    free(d->diag2);
}

static int tree_setup(int64_t n, int32_t leaf, int32_t group, const double *x, const double *m,
                      tree_data *d)
{
    memset(d, 0, sizeof *d);
    if (group < leaf)
        return -1;
    d->nn = oracle_tree_nodes(n, leaf, NULL);
    if (d->nn < 1)
        return -1;
    d->nodes = (int64_t *)malloc((size_t)d->nn * 4 * sizeof(int64_t));
    d->group_node = (int64_t *)malloc((size_t)d->nn * sizeof(int64_t));
    d->mass = (double *)malloc((size_t)d->nn * sizeof(double));
    d->com = (double *)malloc((size_t)d->nn * 3 * sizeof(double));
    d->lo = (double *)malloc((size_t)d->nn * 3 * sizeof(double));
    d->hi = (double *)malloc((size_t)d->nn * 3 * sizeof(double));
    d->diag2 = (double *)malloc((size_t)d->nn * sizeof(double));
    if (!d->nodes || !d->group_node || !d->mass || !d->com || !d->lo || !d->hi || !d->diag2) {
        tree_free(d);
        return -1;
    }
    oracle_tree_nodes(n, leaf, d->nodes);
    d->ngroups = 0;
    tree_groups_rec(d->nodes, 0, group, d->group_node, &d->ngroups);
    return oracle_tree_moments(n, leaf, x, m, d->mass, d->com, d->lo, d->hi, d->diag2);
}

/* Number of groups (see above), or -1 on bad arguments. */
int64_t oracle_tree_num_groups(int64_t n, int32_t leaf, int32_t group)
{
    if (n < 1 || leaf < 1 || group < leaf)
        return -1;
    const int64_t nn = oracle_tree_nodes(n, leaf, NULL);
    int64_t *nodes = (int64_t *)malloc((size_t)nn * 4 * sizeof(int64_t));
    if (!nodes)
        return -1;
    oracle_tree_nodes(n, leaf, nodes);
    int64_t cnt = 0;
    tree_groups_rec(nodes, 0, group, NULL, &cnt);
    free(nodes);
    return cnt;
}

/* Interaction lists of every group, in walk order.  group_id: [ngroups] node
 * id of each group (may be NULL).  far_cnt/near_cnt: [ngroups].  far/near: concatenated lists in group order (NULL to count
 * only; capacities far_cap/near_cap).  Returns 0, or -1 on bad arguments or a
 * list longer than its capacity. */
int oracle_tree_lists(int64_t n, int32_t leaf, int32_t group, const double *x, const double *m,
                      double theta, int64_t *group_id, int64_t *far_cnt, int64_t *near_cnt, int32_t *far,
                      int64_t far_cap, int32_t *near, int64_t near_cap)
{
    if (!(theta >= 0.0) || !far_cnt || !near_cnt)
        return -1;
    tree_data d;
    if (tree_setup(n, leaf, group, x, m, &d) != 0)
        return -1;
    if (group_id)
        memcpy(group_id, d.group_node, (size_t)d.ngroups * sizeof(int64_t));
    tree_ctx t = {d.nodes, d.com, d.lo, d.hi, d.diag2, theta * theta};
    int64_t of = 0, on = 0;
    int rc = 0;
    for (int64_t g = 0; g < d.ngroups; ++g) {
        int64_t nf = 0, nnr = 0;
        tree_walk_rec(&t, 0, d.group_node[g], NULL, &nf, NULL, &nnr);
        far_cnt[g] = nf;
        near_cnt[g] = nnr;
        if (far || near) {
            if (of + nf > far_cap || on + nnr > near_cap) {
                rc = -1;
                break;
            }
            int64_t a = 0, b = 0;
            tree_walk_rec(&t, 0, d.group_node[g], far ? far + of : NULL, &a, near ? near + on : NULL, &b);
        }
        of += nf;
        on += nnr;
    }
    tree_free(&d);
    return rc;
}

/* ---------------------------------------------------------------------------
 * Pseudo-particle multipoles (Makino, J. Comput. Phys. 151, 1999: the
 * paper's reference [20], cited in Section VI for the O(N) FMM).
 *
 * Outside a cell the potential of its bodies is the multipole series
 *   phi(R) = -G sum_i m_i sum_l |r_i|^l / |R|^(l+1) P_l(cos angle(r_i, R)),
 * r_i = x_i - com, R measured from com.  The method replaces the bodies by K
 * point masses q_j at com + a s_j (unit vectors s_j, radius a) whose series
 * is the same for l = 0..p:
 *   q_j = sum_i m_i sum_{l=0..p} (2l+1)/K (|r_i|/a)^l P_l(cos angle(r_i, s_j)).
 * By the addition theorem of the Legendre polynomials this holds whenever
 * the mean of every polynomial of degree <= 2p over the K directions equals
 * its mean over the unit sphere.  Order p = 2 here, with K = 12 directions,
 * the vertices of the icosahedron (a spherical 5-design).  With
 * c_j = s_j . r_i the terms are written without dividing by |r_i|:
 *   l = 0: 1,   l = 1: c_j / a,   l = 2: (3 c_j^2 - |r_i|^2) / (2 a^2).
 * Readings of this library (the paper fixes none of them):
 *   directions  (0, +-1, +-g), (+-1, +-g, 0), (+-g, 0, +-1) divided by
 *               sqrt(1 + g^2), g = (1 + sqrt 5) / 2; j = 0..11 in that order,
 *               the sign pairs of each triple in the order (+,+), (+,-),
 *               (-,+), (-,-).
 *   centre      the cell's FP64 centre of mass (tree moments above).
 *   radius      a = sqrt(diag2) / 2, half the cell's box diagonal; when a = 0
 *               the l >= 1 terms are dropped (q_j = M / 12).
 *   sums        over the cell's bodies in position order, Neumaier-compensated.
 *   force       an accepted cell acts as its 12 pseudo-particles, j = 0..11,
 *               with the softened pair law of the bodies.
 * ------------------------------------------------------------------------- */
#define PSEUDO_K 12

static void pseudo_dirs(double s[PSEUDO_K][3])
{
    const double g = 0.5 * (1.0 + sqrt(5.0));
    const double inv = 1.0 / sqrt(1.0 + g * g);
    static const double sg[4][2] = {{1, 1}, {1, -1}, {-1, 1}, {-1, -1}};
    for (int k = 0; k < 4; ++k) {
        const double u = sg[k][0], v = sg[k][1];
        /* (0, +-1, +-g) */
        s[k][0] = 0.0;
        s[k][1] = u * inv;
        s[k][2] = v * g * inv;
        /* (+-1, +-g, 0) */
        s[4 + k][0] = u * inv;
        s[4 + k][1] = v * g * inv;
        s[4 + k][2] = 0.0;
        /* (+-g, 0, +-1) */
        s[8 + k][0] = u * g * inv;
        s[8 + k][1] = 0.0;
        s[8 + k][2] = v * inv;
    }
}

/* The 12 unit directions, [12][3]. */
void oracle_pseudo_dirs(double *out)
{
    double s[PSEUDO_K][3];
    pseudo_dirs(s);
    memcpy(out, s, sizeof(s));
}

/* Pseudo-particles of every node from its bodies: out [nn][12][4] =
 * (x, y, z, q).  d holds the node table and the monopole moments. */
static void tree_pseudo_fill(const tree_data *d, const double *x, const double *m, double *out)
{
    double s[PSEUDO_K][3];
    pseudo_dirs(s);
    int64_t c;
#pragma omp parallel for schedule(dynamic, 64)
    for (c = 0; c < d->nn; ++c) {
        const double *cm = d->com + 3 * c;
        const double a = 0.5 * sqrt(d->diag2[c]);
        for (int j = 0; j < PSEUDO_K; ++j) {
            nsum q = {0, 0};
            for (int64_t i = d->nodes[4 * c]; i < d->nodes[4 * c + 1]; ++i) {
                const double rx = x[3 * i] - cm[0], ry = x[3 * i + 1] - cm[1], rz = x[3 * i + 2] - cm[2];
                double t = 1.0 / PSEUDO_K;
                if (a > 0.0) {
                    const double cj = (s[j][0] * rx + s[j][1] * ry) + s[j][2] * rz;
                    const double r2 = (rx * rx + ry * ry) + rz * rz;
                    t = t + 3.0 / PSEUDO_K * (cj / a);
                    t = t + 5.0 / PSEUDO_K * ((3.0 * cj * cj - r2) / (2.0 * a * a));
                }
                nsum_add(&q, m[i] * t);
            }
            double *o = out + 4 * (PSEUDO_K * c + j);
            o[0] = cm[0] + a * s[j][0];
            o[1] = cm[1] + a * s[j][1];
            o[2] = cm[2] + a * s[j][2];
            o[3] = nsum_val(&q);
        }
    }
}

/* Pseudo-particles of every node (ORB positions): out [nn][12][4] =
 * (x, y, z, q).  Returns 0, or -1 on bad arguments. */
int oracle_tree_pseudo(int64_t n, int32_t leaf, const double *x, const double *m, double *out)
{
    tree_data d;
    if (tree_setup(n, leaf, leaf, x, m, &d) != 0)
        return -1;
    tree_pseudo_fill(&d, x, m, out);
    tree_free(&d);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Quadrupole cells evaluated directly.  The same expansion through l = 2,
 * written with the traceless quadrupole tensor of the cell about its centre
 * of mass,
 *   Q = sum_i m_i (3 r_i r_i^T - |r_i|^2 I),   r_i = x_i - com,
 * is, at a target at offset d = x - com,
 *   phi = -G (M / s + d.Q.d / (2 s^5)),
 *   a   =  G (-M d / s^3 + Q d / s^5 - 5 (d.Q.d) d / (2 s^7)),
 * a = -grad phi, with the softened distance s^2 = |d|^2 + eps^2 in place of
 * |d| (this library's reading: the expansion of the softened monopole law,
 * differentiated as written).  Q is summed over the cell's bodies in position
 * order, Neumaier-compensated.
 * ------------------------------------------------------------------------- */
static void tree_quad_fill(const tree_data *d, const double *x, const double *m, double *out)
{
    int64_t c;
#pragma omp parallel for schedule(dynamic, 64)
    for (c = 0; c < d->nn; ++c) {
        const double *cm = d->com + 3 * c;
        nsum q[6] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}};
        for (int64_t i = d->nodes[4 * c]; i < d->nodes[4 * c + 1]; ++i) {
            const double r[3] = {x[3 * i] - cm[0], x[3 * i + 1] - cm[1], x[3 * i + 2] - cm[2]};
            const double r2 = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
            nsum_add(&q[0], m[i] * (3.0 * r[0] * r[0] - r2));
            nsum_add(&q[1], m[i] * (3.0 * r[1] * r[1] - r2));
            nsum_add(&q[2], m[i] * (3.0 * r[2] * r[2] - r2));
            nsum_add(&q[3], m[i] * (3.0 * r[0] * r[1]));
            nsum_add(&q[4], m[i] * (3.0 * r[0] * r[2]));
            nsum_add(&q[5], m[i] * (3.0 * r[1] * r[2]));
        }
        for (int k = 0; k < 6; ++k)
            out[6 * c + k] = nsum_val(&q[k]);
    }
}

/* Traceless quadrupole of every node (ORB positions): out [nn][6] =
 * (Qxx, Qyy, Qzz, Qxy, Qxz, Qyz).  Returns 0, or -1 on bad arguments. */
int oracle_tree_quad(int64_t n, int32_t leaf, const double *x, const double *m, double *out)
{
    tree_data d;
    if (tree_setup(n, leaf, leaf, x, m, &d) != 0)
        return -1;
    tree_quad_fill(&d, x, m, out);
    tree_free(&d);
    return 0;
}

/* Third-order local expansion of the potential sum of one quadrupole cell
 * (mass M, centre of mass cm, traceless Q as (xx, yy, zz, xy, xz, yz))
 * about the point zg, formulas above; the 20 coefficients
 *   L[0] = P0, L[1..3] = p, L[4..9] = K (xx, yy, zz, xy, xz, yz),
 *   L[10..19] = T (xxx, yyy, zzz, xxy, xxz, xyy, yyz, xzz, yzz, xyz)
 * are added to the running sums L. */
static const int local_tt[10][3] = {{0, 0, 0}, {1, 1, 1}, {2, 2, 2}, {0, 0, 1}, {0, 0, 2},
                                    {0, 1, 1}, {1, 1, 2}, {0, 2, 2}, {1, 2, 2}, {0, 1, 2}};

static void local_m2l_add(nsum *L, const double *zg, const double *cm, double M, const double *Qv, double eps2)
{
    const double Q[3][3] = {{Qv[0], Qv[3], Qv[4]}, {Qv[3], Qv[1], Qv[5]}, {Qv[4], Qv[5], Qv[2]}};
    const double r[3] = {zg[0] - cm[0], zg[1] - cm[1], zg[2] - cm[2]};
    const double s2 = ((r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]) + eps2;
    const double s1 = 1.0 / sqrt(s2);
    const double s3 = s1 / s2, s5 = s3 / s2, s7 = s5 / s2, s9 = s7 / s2, s11 = s9 / s2;
    double qr[3];
    for (int k = 0; k < 3; ++k)
        qr[k] = (Q[k][0] * r[0] + Q[k][1] * r[1]) + Q[k][2] * r[2];
    const double rqr = (r[0] * qr[0] + r[1] * qr[1]) + r[2] * qr[2];
    nsum_add(&L[0], M * s1 + 0.5 * rqr * s5);
    for (int k = 0; k < 3; ++k)
        nsum_add(&L[1 + k], -M * r[k] * s3 - 2.5 * rqr * r[k] * s7 + qr[k] * s5);
    /* K in the order xx, yy, zz, xy, xz, yz */
    static const int kk[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
    for (int u = 0; u < 6; ++u) {
        const int k = kk[u][0], l = kk[u][1];
        const double dkl = k == l ? 1.0 : 0.0;
        const double v = M * (3.0 * r[k] * r[l] * s5 - dkl * s3) + 17.5 * rqr * r[k] * r[l] * s9 -
                         2.5 * (2.0 * qr[k] * r[l] + 2.0 * qr[l] * r[k] + dkl * rqr) * s7 +
                         Q[k][l] * s5;
        nsum_add(&L[4 + u], v);
    }
    /* T in the order of local_tt */
    for (int u = 0; u < 10; ++u) {
        const int k = local_tt[u][0], l = local_tt[u][1], m2 = local_tt[u][2];
        const double dkl = k == l ? 1.0 : 0.0, dkm = k == m2 ? 1.0 : 0.0, dlm = l == m2 ? 1.0 : 0.0;
        const double rrr = r[k] * r[l] * r[m2];
        const double dr = dkl * r[m2] + dkm * r[l] + dlm * r[k];
        const double v = M * (-15.0 * rrr * s7 + 3.0 * dr * s5) - 157.5 * rqr * rrr * s11 +
                         35.0 * (qr[k] * r[l] * r[m2] + qr[l] * r[k] * r[m2] + qr[m2] * r[k] * r[l]) * s9 +
                         17.5 * rqr * dr * s9 -
                         5.0 * (Q[k][l] * r[m2] + Q[k][m2] * r[l] + Q[l][m2] * r[k] + qr[k] * dlm +
                                qr[l] * dkm + qr[m2] * dkl) * s7;
        nsum_add(&L[10 + u], v);
    }
}

/* The full symmetric K (3x3) and T (3x3x3) of the 20 stored coefficients. */
static void local_tensors(const double *c, double K[3][3], double T3[3][3][3])
{
    K[0][0] = c[4];
    K[1][1] = c[5];
    K[2][2] = c[6];
    K[0][1] = K[1][0] = c[7];
    K[0][2] = K[2][0] = c[8];
    K[1][2] = K[2][1] = c[9];
    static const int pm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    for (int u = 0; u < 10; ++u) {
        const int *a3 = local_tt[u];
        for (int w = 0; w < 6; ++w)
            T3[a3[pm[w][0]]][a3[pm[w][1]]][a3[pm[w][2]]] = c[10 + u];
    }
}

/* L2P: the expansion c at offset y from its centre.  Adds the gradient
 * p + K y + T(y, y) / 2 to (ax, ay, az) and the value P0 + p.y + y.K.y / 2 +
 * T(y, y, y) / 6 to ph (acceleration = G times the former, potential = -G
 * times the latter). */
static void local_l2p_add(const double *c, const double *y, nsum *ax, nsum *ay, nsum *az, nsum *ph)
{
    double K[3][3], T3[3][3][3];
    local_tensors(c, K, T3);
    double ky[3], tyy[3];
    for (int k = 0; k < 3; ++k) {
        ky[k] = (K[k][0] * y[0] + K[k][1] * y[1]) + K[k][2] * y[2];
        tyy[k] = 0.0;
        for (int l = 0; l < 3; ++l)
            for (int m2 = 0; m2 < 3; ++m2)
                tyy[k] += T3[k][l][m2] * y[l] * y[m2];
    }
    nsum_add(ax, c[1] + ky[0] + 0.5 * tyy[0]);
    nsum_add(ay, c[2] + ky[1] + 0.5 * tyy[1]);
    nsum_add(az, c[3] + ky[2] + 0.5 * tyy[2]);
    const double py = (c[1] * y[0] + c[2] * y[1]) + c[3] * y[2];
    const double yky = (y[0] * ky[0] + y[1] * ky[1]) + y[2] * ky[2];
    const double ytyy = (y[0] * tyy[0] + y[1] * tyy[1]) + y[2] * tyy[2];
    nsum_add(ph, c[0] + py + 0.5 * yky + ytyy / 6.0);
}

/* One quadrupole cell (mass M at com cm, traceless tensor Qv = xx, yy, zz,
 * xy, xz, yz) at the point (xi, yi, zi), d = x - com, s^2 = |d|^2 + eps^2:
 *   phi-sum += M/s + d.Q.d / (2 s^5),
 *   a-sum   += -M d / s^3 + Q d / s^5 - 5 (d.Q.d) d / (2 s^7)
 * (the expansion of the cell's potential through l = 2 with the softened
 * distance in place of |d|; the caller scales by G and the sign). */
static void quad_cell_add(double xi, double yi, double zi, const double *cm, double M, const double *Q,
                          double eps2, nsum *ax, nsum *ay, nsum *az, nsum *ph)
{
    const double dv[3] = {xi - cm[0], yi - cm[1], zi - cm[2]};
    const double s2 = ((dv[0] * dv[0] + dv[1] * dv[1]) + dv[2] * dv[2]) + eps2;
    const double s = sqrt(s2);
    const double qd[3] = {(Q[0] * dv[0] + Q[3] * dv[1]) + Q[4] * dv[2],
                          (Q[3] * dv[0] + Q[1] * dv[1]) + Q[5] * dv[2],
                          (Q[4] * dv[0] + Q[5] * dv[1]) + Q[2] * dv[2]};
    const double dqd = (dv[0] * qd[0] + dv[1] * qd[1]) + dv[2] * qd[2];
    const double s3 = s2 * s, s5 = s3 * s2, s7 = s5 * s2;
    for (int k = 0; k < 3; ++k) {
        nsum *ak = k == 0 ? ax : (k == 1 ? ay : az);
        nsum_add(ak, -M * dv[k] / s3);
        nsum_add(ak, qd[k] / s5);
        nsum_add(ak, -2.5 * dqd * dv[k] / s7);
    }
    nsum_add(ph, M / s);
    nsum_add(ph, 0.5 * dqd / s5);
}

/* Tree force and potential on targets (ORB positions; NULL = all n).
 * acc: [ntarg][3], pot: [ntarg].  cells 0: an accepted cell acts as one body
 * (M at com); 2: as its 12 pseudo-particles; 3: through its quadrupole
 * expansion (above).  Neumaier-compensated FP64 sums over the far cells in
 * list order (pseudo-particles j = 0..11 within a cell), then the near
 * bodies in list order. */
int oracle_tree_accel_cells(int64_t n, int32_t leaf, int32_t group, const double *x, const double *m,
                            double G, double eps, double theta, int32_t cells, int64_t ntarg,
                            const int64_t *targets, double *acc, double *pot)
{
    if (!(theta >= 0.0) || cells < 0 || cells == 1 || cells > 4)
        return -1;
    tree_data d;
    if (tree_setup(n, leaf, group, x, m, &d) != 0)
        return -1;
    double *pp = NULL;
    if (cells >= 2) {
        const size_t per = cells == 2 ? PSEUDO_K * 4 : 6;
        pp = (double *)malloc((size_t)d.nn * per * sizeof(double));
        if (!pp) {
            tree_free(&d);
            return -1;
        }
        if (cells == 2)
            tree_pseudo_fill(&d, x, m, pp);
        else
            tree_quad_fill(&d, x, m, pp);
    }
    tree_ctx tc = {d.nodes, d.com, d.lo, d.hi, d.diag2, theta * theta};
    /* group of every position */
    int64_t *gof = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!gof) {
        free(pp);
        tree_free(&d);
        return -1;
    }
    for (int64_t q = 0; q < d.ngroups; ++q)
        for (int64_t p = d.nodes[4 * d.group_node[q]]; p < d.nodes[4 * d.group_node[q] + 1]; ++p)
            gof[p] = d.group_node[q];
    const double eps2 = eps * eps;
    int bad = 0;
    int64_t t;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
    for (t = 0; t < ntarg; ++t) {
        const int64_t i = targets ? targets[t] : t;
        const int64_t g = gof[i];
        int64_t nl = 0, nf = 0, nnr = 0;
        if (cells == 4)
            tree_walk_local_rec(&tc, 0, g, NULL, &nl, NULL, &nf, NULL, &nnr);
        else
            tree_walk_rec(&tc, 0, g, NULL, &nf, NULL, &nnr);
        int32_t *loc = (int32_t *)malloc((size_t)(nl + 1) * sizeof(int32_t));
        int32_t *far = (int32_t *)malloc((size_t)(nf + 1) * sizeof(int32_t));
        int32_t *near = (int32_t *)malloc((size_t)(nnr + 1) * sizeof(int32_t));
        if (!loc || !far || !near) {
            free(loc);
            free(far);
            free(near);
            bad = 1;
            continue;
        }
        int64_t a = 0, b = 0, e = 0;
        if (cells == 4)
            tree_walk_local_rec(&tc, 0, g, loc, &e, far, &a, near, &b);
        else
            tree_walk_rec(&tc, 0, g, far, &a, near, &b);
        const double xi = x[3 * i], yi = x[3 * i + 1], zi = x[3 * i + 2];
        nsum ax = {0, 0}, ay = {0, 0}, az = {0, 0}, ph = {0, 0};
        if (nl > 0) {
            /* M2L over the local list, then L2P at this target */
            const double *zg = d.com + 3 * g;
            nsum L[20];
            for (int k = 0; k < 20; ++k)
                L[k] = (nsum){0, 0};
            for (int64_t q = 0; q < nl; ++q) {
                const int64_t c = loc[q];
                local_m2l_add(L, zg, d.com + 3 * c, d.mass[c], pp + 6 * c, eps2);
            }
            double c[20];
            for (int k = 0; k < 20; ++k)
                c[k] = nsum_val(&L[k]);
            const double y[3] = {xi - zg[0], yi - zg[1], zi - zg[2]};
            local_l2p_add(c, y, &ax, &ay, &az, &ph);
        }
        for (int64_t q = 0; q < nf + nnr; ++q) {
            const int64_t c = q < nf ? far[q] : near[q - nf];
            if (q < nf && cells >= 3) {
                quad_cell_add(xi, yi, zi, d.com + 3 * c, d.mass[c], pp + 6 * c, eps2, &ax, &ay, &az, &ph);
                continue;
            }
            int64_t jb, je;
            if (q < nf) {
                jb = 0;
                je = cells == 0 ? 1 : PSEUDO_K;
            } else {
                jb = d.nodes[4 * c];
                je = d.nodes[4 * c + 1];
            }
            for (int64_t j = jb; j < je; ++j) {
                const double *xj;
                double mj;
                if (q >= nf) {
                    if (j == i)
                        continue;
                    xj = x + 3 * j;
                    mj = m[j];
                } else if (cells == 0) {
                    xj = d.com + 3 * c;
                    mj = d.mass[c];
                } else {
                    xj = pp + 4 * (PSEUDO_K * c + j);
                    mj = xj[3];
                }
                const double dx = xj[0] - xi;
                const double dy = xj[1] - yi;
                const double dz = xj[2] - zi;
                const double r2 = ((dx * dx + dy * dy) + dz * dz) + eps2;
                const double r = sqrt(r2);
                const double w = 1.0 / (r2 * r);
                const double mw = mj * w;
                nsum_add(&ax, mw * dx);
                nsum_add(&ay, mw * dy);
                nsum_add(&az, mw * dz);
                nsum_add(&ph, mj / r);
            }
        }
        free(loc);
        free(far);
        free(near);
        if (acc) {
            acc[3 * t] = G * nsum_val(&ax);
            acc[3 * t + 1] = G * nsum_val(&ay);
            acc[3 * t + 2] = G * nsum_val(&az);
        }
        if (pot)
            pot[t] = -G * nsum_val(&ph);
    }
    free(gof);
    free(pp);
    tree_free(&d);
    return bad ? -1 : 0;
}

/* Lists of the local-expansion walk for every group, in walk order:
 * loc/far/near concatenated in group order with capacities; the counts as
 * in oracle_tree_local_counts.  Returns 0, or -1 on bad arguments or a list
 * longer than its capacity. */
int oracle_tree_local_lists(int64_t n, int32_t leaf, int32_t group, const double *x, const double *m,
                            double theta, int64_t *loc_cnt, int64_t *far_cnt, int64_t *near_cnt, int32_t *loc,
                            int64_t loc_cap, int32_t *far, int64_t far_cap, int32_t *near, int64_t near_cap)
{
    if (!(theta >= 0.0))
        return -1;
    tree_data d;
    if (tree_setup(n, leaf, group, x, m, &d) != 0)
        return -1;
    tree_ctx tc = {d.nodes, d.com, d.lo, d.hi, d.diag2, theta * theta};
    int64_t ol = 0, of = 0, on = 0;
    int rc = 0;
    for (int64_t q = 0; q < d.ngroups && rc == 0; ++q) {
        int64_t a = 0, b = 0, e = 0;
        tree_walk_local_rec(&tc, 0, d.group_node[q], NULL, &e, NULL, &a, NULL, &b);
        loc_cnt[q] = e;
        far_cnt[q] = a;
        near_cnt[q] = b;
        if (ol + e > loc_cap || of + a > far_cap || on + b > near_cap) {
            rc = -1;
            break;
        }
        int64_t a2 = 0, b2 = 0, e2 = 0;
        tree_walk_local_rec(&tc, 0, d.group_node[q], loc + ol, &e2, far + of, &a2, near + on, &b2);
        ol += e;
        of += a;
        on += b;
    }
    tree_free(&d);
    return rc;
}

/* Per-group list sizes of the local-expansion walk: loc_cnt, far_cnt,
 * near_cnt [ngroups].  Returns 0, or -1 on bad arguments. */
int oracle_tree_local_counts(int64_t n, int32_t leaf, int32_t group, const double *x, const double *m,
                             double theta, int64_t *loc_cnt, int64_t *far_cnt, int64_t *near_cnt)
{
    if (!(theta >= 0.0))
        return -1;
    tree_data d;
    if (tree_setup(n, leaf, group, x, m, &d) != 0)
        return -1;
    tree_ctx tc = {d.nodes, d.com, d.lo, d.hi, d.diag2, theta * theta};
    for (int64_t q = 0; q < d.ngroups; ++q) {
        int64_t a = 0, b = 0, e = 0;
        tree_walk_local_rec(&tc, 0, d.group_node[q], NULL, &e, NULL, &a, NULL, &b);
        loc_cnt[q] = e;
        far_cnt[q] = a;
        near_cnt[q] = b;
    }
    tree_free(&d);
    return 0;
}

/* The monopole tree force (cells 0 of the above). */
int oracle_tree_accel(int64_t n, int32_t leaf, int32_t group, const double *x, const double *m, double G,
                      double eps, double theta, int64_t ntarg, const int64_t *targets, double *acc,
                      double *pot)
{
    return oracle_tree_accel_cells(n, leaf, group, x, m, G, eps, theta, 0, ntarg, targets, acc, pot);
}

/* ---------------------------------------------------------------------------
 * Multi-level fast multipole method on the ORB hierarchy: the O(N) method
 * Section VI names (citing its reference [20]) as the way beyond the tree
 * code, built from the quadrupole cells and third-order local expansions
 * above.  Readings of this library (the paper gives no formulas):
 *   cells     every node carries its quadrupole expansion about its centre
 *             of mass (oracle_tree_quad); every node's local expansion is
 *             about the same centre, z_A = com_A.
 *   MAC       nodes A (targets) and B (sources) interact through M2L iff
 *             they share no body and diag2_A + diag2_B < theta^2
 *             |com_A - com_B|^2 (the group local test, now between any two
 *             nodes).
 *   traversal interact(A, B) from (root, root):
 *               MAC(A, B)          -> B joins the M2L list of A
 *               A a leaf that the tree code's opening test accepts B for
 *               (diag2_B < theta^2 D2, D2 from com_B to A's box; see
 *               tree_accept)      -> B joins the M2P list of A
 *               A, B both leaves   -> B joins the P2P list of A
 *               B a leaf, or A not a leaf with diag2_A >= diag2_B
 *                                  -> interact(A.left, B), interact(A.right, B)
 *               else               -> interact(A, B.left), interact(A, B.right)
 *             Every ordered pair of distinct bodies (i, j) is then counted
 *             once: through the M2L entry of an ancestor-or-self of i's
 *             leaf whose source contains j, or through the M2P or P2P entry
 *             of i's leaf whose source contains j.  The M2P case keeps a
 *             leaf whose box is large against its distance to the rest (a
 *             few bodies far out in a halo) from failing the MAC against
 *             every node and pairing with every leaf.
 *   M2L       local_m2l_add, summed over a node's list in traversal order.
 *   L2L       a node's total expansion = its own M2L sum + its parent's
 *             total re-expanded about its centre (local_shift: a cubic
 *             re-expanded exactly), coefficient by coefficient.
 *   L2P, M2P, P2P  per body of a leaf: the leaf's total expansion at the
 *             body (local_l2p_add), then its M2P cells in list order as
 *             quadrupole cells (quad_cell_add), then the P2P source leaves
 *             in list order body by body, skipping the body itself;
 *             Neumaier sums.
 * theta = 0 gives no M2L entry, so the result is the direct sum.
 * ------------------------------------------------------------------------- */

/* Re-expands the cubic c about its centre z as a cubic about z + dz (exact
 * up to rounding): with f(y) = P0 + p.y + y.K.y/2 + T(y,y,y)/6,
 *   P0' = P0 + p.dz + dz.K.dz/2 + T(dz,dz,dz)/6,  p' = p + K dz + T(dz,dz)/2,
 *   K'  = K + T dz,  T' = T. */
void oracle_local_shift(const double *c, const double *dz, double *out)
{
    double K[3][3], T3[3][3][3];
    local_tensors(c, K, T3);
    double kd[3], td[3][3], tdd[3];
    for (int k = 0; k < 3; ++k) {
        kd[k] = (K[k][0] * dz[0] + K[k][1] * dz[1]) + K[k][2] * dz[2];
        for (int l = 0; l < 3; ++l)
            td[k][l] = (T3[k][l][0] * dz[0] + T3[k][l][1] * dz[1]) + T3[k][l][2] * dz[2];
        tdd[k] = (td[k][0] * dz[0] + td[k][1] * dz[1]) + td[k][2] * dz[2];
    }
    const double pd = (c[1] * dz[0] + c[2] * dz[1]) + c[3] * dz[2];
    const double dkd = (dz[0] * kd[0] + dz[1] * kd[1]) + dz[2] * kd[2];
    const double dtdd = (dz[0] * tdd[0] + dz[1] * tdd[1]) + dz[2] * tdd[2];
    out[0] = c[0] + pd + 0.5 * dkd + dtdd / 6.0;
    for (int k = 0; k < 3; ++k)
        out[1 + k] = c[1 + k] + kd[k] + 0.5 * tdd[k];
    out[4] = c[4] + td[0][0];
    out[5] = c[5] + td[1][1];
    out[6] = c[6] + td[2][2];
    out[7] = c[7] + td[0][1];
    out[8] = c[8] + td[0][2];
    out[9] = c[9] + td[1][2];
    for (int u = 10; u < 20; ++u)
        out[u] = c[u];
}

typedef struct {
    int32_t *a, *b;
    int64_t n, cap;
    int fail;
} fmm_pairs;

static void fmm_push(fmm_pairs *l, int64_t a, int64_t b)
{
    if (l->fail)
        return;
    if (l->n == l->cap) {
        const int64_t cap = l->cap ? 2 * l->cap : 1024;
        int32_t *na = (int32_t *)realloc(l->a, (size_t)cap * sizeof(int32_t));
        if (na)
            l->a = na;
        int32_t *nb = (int32_t *)realloc(l->b, (size_t)cap * sizeof(int32_t));
        if (nb)
            l->b = nb;
        if (!na || !nb) {
            l->fail = 1;
            return;
        }
        l->cap = cap;
    }
    l->a[l->n] = (int32_t)a;
    l->b[l->n] = (int32_t)b;
    ++l->n;
}

typedef struct {
    const tree_data *d;
    tree_ctx tc; /* the tree code's opening test on the same moments */
    double theta2;
    fmm_pairs m2l, m2p, p2p;
} fmm_ctx;

static int fmm_mac(const fmm_ctx *f, int64_t a, int64_t b)
{
    const tree_data *d = f->d;
    if (tree_overlap(d->nodes, a, b))
        return 0;
    const double dx = d->com[3 * a] - d->com[3 * b];
    const double dy = d->com[3 * a + 1] - d->com[3 * b + 1];
    const double dz = d->com[3 * a + 2] - d->com[3 * b + 2];
    const double dist2 = (dx * dx + dy * dy) + dz * dz;
    return d->diag2[a] + d->diag2[b] < f->theta2 * dist2;
}

static void fmm_interact(fmm_ctx *f, int64_t a, int64_t b)
{
    if (fmm_mac(f, a, b)) {
        fmm_push(&f->m2l, a, b);
        return;
    }
    const int64_t *nodes = f->d->nodes;
    const int64_t al = nodes[4 * a + 2], ar = nodes[4 * a + 3];
    const int64_t bl = nodes[4 * b + 2], br = nodes[4 * b + 3];
    if (al < 0 && tree_accept(&f->tc, b, a)) {
        fmm_push(&f->m2p, a, b);
        return;
    }
    if (al < 0 && bl < 0) {
        fmm_push(&f->p2p, a, b);
        return;
    }
    if (bl < 0 || (al >= 0 && f->d->diag2[a] >= f->d->diag2[b])) {
        fmm_interact(f, al, b);
        fmm_interact(f, ar, b);
    } else {
        fmm_interact(f, a, bl);
        fmm_interact(f, a, br);
    }
}

/* Stable grouping of a pair list by target node: cnt[nn] per target,
 * start[nn] offsets, src[] the sources in traversal order per target. */
static int fmm_by_target(const fmm_pairs *l, int64_t nn, int64_t *cnt, int64_t *start, int32_t *src)
{
    for (int64_t k = 0; k < nn; ++k)
        cnt[k] = 0;
    for (int64_t q = 0; q < l->n; ++q)
        ++cnt[l->a[q]];
    int64_t o = 0;
    for (int64_t k = 0; k < nn; ++k) {
        start[k] = o;
        o += cnt[k];
    }
    int64_t *fill = (int64_t *)malloc((size_t)nn * sizeof(int64_t));
    if (!fill)
        return -1;
    memcpy(fill, start, (size_t)nn * sizeof(int64_t));
    for (int64_t q = 0; q < l->n; ++q)
        src[fill[l->a[q]]++] = l->b[q];
    free(fill);
    return 0;
}

static int fmm_run(int64_t n, int32_t leaf, const double *x, const double *m, double theta, tree_data *d,
                   fmm_ctx *f)
{
    memset(f, 0, sizeof *f);
    if (!(theta >= 0.0) || tree_setup(n, leaf, leaf, x, m, d) != 0)
        return -1;
    f->d = d;
    f->theta2 = theta * theta;
    f->tc = (tree_ctx){d->nodes, d->com, d->lo, d->hi, d->diag2, f->theta2};
    fmm_interact(f, 0, 0);
    if (f->m2l.fail || f->m2p.fail || f->p2p.fail) {
        tree_free(d);
        return -1;
    }
    return 0;
}

static void fmm_ctx_free(fmm_ctx *f)
{
    free(f->m2l.a);
    free(f->m2l.b);
    free(f->m2p.a);
    free(f->m2p.b);
    free(f->p2p.a);
    free(f->p2p.b);
}

/* The FMM's lists grouped by target node (node ids in preorder):
 * m2l_cnt/m2p_cnt/p2p_cnt [nn]; m2l/m2p/p2p the source node ids of every
 * target in traversal order, targets in node order (NULL to count only;
 * capacities m2l_cap/m2p_cap/p2p_cap).  Returns 0, or -1 on bad arguments or
 * a list longer than its capacity. */
int oracle_fmm_lists(int64_t n, int32_t leaf, const double *x, const double *m, double theta, int64_t *m2l_cnt,
                     int64_t *m2p_cnt, int64_t *p2p_cnt, int32_t *m2l, int64_t m2l_cap, int32_t *m2p,
                     int64_t m2p_cap, int32_t *p2p, int64_t p2p_cap)
{
    tree_data d;
    fmm_ctx f;
    if (!m2l_cnt || !m2p_cnt || !p2p_cnt || fmm_run(n, leaf, x, m, theta, &d, &f) != 0)
        return -1;
    int rc = 0;
    int64_t *start = (int64_t *)malloc((size_t)d.nn * sizeof(int64_t));
    int32_t *tmp = (int32_t *)malloc((size_t)(f.m2l.n + f.m2p.n + f.p2p.n + 1) * sizeof(int32_t));
    if (!start || !tmp)
        rc = -1;
    const fmm_pairs *lists[3] = {&f.m2l, &f.m2p, &f.p2p};
    int64_t *cnts[3] = {m2l_cnt, m2p_cnt, p2p_cnt};
    int32_t *outs[3] = {m2l, m2p, p2p};
    const int64_t caps[3] = {m2l_cap, m2p_cap, p2p_cap};
    for (int w = 0; w < 3 && rc == 0; ++w) {
        rc |= fmm_by_target(lists[w], d.nn, cnts[w], start, tmp);
        if (rc == 0 && outs[w]) {
            if (lists[w]->n > caps[w])
                rc = -1;
            else
                memcpy(outs[w], tmp, (size_t)lists[w]->n * sizeof(int32_t));
        }
    }
    free(start);
    free(tmp);
    fmm_ctx_free(&f);
    tree_free(&d);
    return rc;
}

/* FMM force and potential on targets (ORB positions; NULL = all n).
 * acc: [ntarg][3], pot: [ntarg].  Returns 0, or -1 on bad arguments. */
int oracle_fmm_accel(int64_t n, int32_t leaf, const double *x, const double *m, double G, double eps,
                     double theta, int64_t ntarg, const int64_t *targets, double *acc, double *pot)
{
    tree_data d;
    fmm_ctx f;
    if (fmm_run(n, leaf, x, m, theta, &d, &f) != 0)
        return -1;
    const int64_t nn = d.nn;
    const double eps2 = eps * eps;
    double *Q = (double *)malloc((size_t)nn * 6 * sizeof(double));
    nsum *own = (nsum *)calloc((size_t)nn * 20, sizeof(nsum));
    double *tot = (double *)malloc((size_t)nn * 20 * sizeof(double));
    int64_t *pcnt = (int64_t *)malloc((size_t)nn * sizeof(int64_t));
    int64_t *pstart = (int64_t *)malloc((size_t)nn * sizeof(int64_t));
    int32_t *psrc = (int32_t *)malloc((size_t)(f.p2p.n + 1) * sizeof(int32_t));
    int64_t *ccnt = (int64_t *)malloc((size_t)nn * sizeof(int64_t));
    int64_t *cstart = (int64_t *)malloc((size_t)nn * sizeof(int64_t));
    int32_t *csrc = (int32_t *)malloc((size_t)(f.m2p.n + 1) * sizeof(int32_t));
    int64_t *leaf_of = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int rc = (Q && own && tot && pcnt && pstart && psrc && ccnt && cstart && csrc && leaf_of) ? 0 : -1;
    if (rc == 0)
        rc = fmm_by_target(&f.p2p, nn, pcnt, pstart, psrc);
    if (rc == 0)
        rc = fmm_by_target(&f.m2p, nn, ccnt, cstart, csrc);
    if (rc == 0) {
        tree_quad_fill(&d, x, m, Q);
        /* M2L in traversal order */
        for (int64_t q = 0; q < f.m2l.n; ++q) {
            const int64_t a = f.m2l.a[q], b = f.m2l.b[q];
            local_m2l_add(own + 20 * a, d.com + 3 * a, d.com + 3 * b, d.mass[b], Q + 6 * b, eps2);
        }
        /* L2L top-down: preorder numbering puts every parent before its
         * children */
        for (int k = 0; k < 20; ++k)
            tot[k] = nsum_val(&own[k]);
        for (int64_t a = 0; a < nn; ++a) {
            const int64_t ch[2] = {d.nodes[4 * a + 2], d.nodes[4 * a + 3]};
            if (ch[0] < 0) {
                for (int64_t p = d.nodes[4 * a]; p < d.nodes[4 * a + 1]; ++p)
                    leaf_of[p] = a;
                continue;
            }
            for (int h = 0; h < 2; ++h) {
                const int64_t c = ch[h];
                const double dz[3] = {d.com[3 * c] - d.com[3 * a], d.com[3 * c + 1] - d.com[3 * a + 1],
                                      d.com[3 * c + 2] - d.com[3 * a + 2]};
                double sh[20];
                oracle_local_shift(tot + 20 * a, dz, sh);
                for (int k = 0; k < 20; ++k)
                    tot[20 * c + k] = nsum_val(&own[20 * c + k]) + sh[k];
            }
        }
        int64_t t;
#pragma omp parallel for schedule(dynamic, 64)
        for (t = 0; t < ntarg; ++t) {
            const int64_t i = targets ? targets[t] : t;
            const int64_t a = leaf_of[i];
            const double *za = d.com + 3 * a;
            const double xi = x[3 * i], yi = x[3 * i + 1], zi = x[3 * i + 2];
            nsum ax = {0, 0}, ay = {0, 0}, az = {0, 0}, ph = {0, 0};
            const double y[3] = {xi - za[0], yi - za[1], zi - za[2]};
            local_l2p_add(tot + 20 * a, y, &ax, &ay, &az, &ph);
            for (int64_t q = cstart[a]; q < cstart[a] + ccnt[a]; ++q) {
                const int64_t b = csrc[q];
                quad_cell_add(xi, yi, zi, d.com + 3 * b, d.mass[b], Q + 6 * b, eps2, &ax, &ay, &az, &ph);
            }
            for (int64_t q = pstart[a]; q < pstart[a] + pcnt[a]; ++q) {
                const int64_t b = psrc[q];
                for (int64_t j = d.nodes[4 * b]; j < d.nodes[4 * b + 1]; ++j) {
                    if (j == i)
                        continue;
                    const double dx = x[3 * j] - xi;
                    const double dy = x[3 * j + 1] - yi;
                    const double dzz = x[3 * j + 2] - zi;
                    const double r2 = ((dx * dx + dy * dy) + dzz * dzz) + eps2;
                    const double r = sqrt(r2);
                    const double w = 1.0 / (r2 * r);
                    const double mw = m[j] * w;
                    nsum_add(&ax, mw * dx);
                    nsum_add(&ay, mw * dy);
                    nsum_add(&az, mw * dzz);
                    nsum_add(&ph, m[j] / r);
                }
            }
            if (acc) {
                acc[3 * t] = G * nsum_val(&ax);
                acc[3 * t + 1] = G * nsum_val(&ay);
                acc[3 * t + 2] = G * nsum_val(&az);
            }
            if (pot)
                pot[t] = -G * nsum_val(&ph);
        }
    }
    free(Q);
    free(own);
    free(tot);
    free(pcnt);
    free(pstart);
    free(psrc);
    free(ccnt);
    free(cstart);
    free(csrc);
    free(leaf_of);
    fmm_ctx_free(&f);
    tree_free(&d);
    return rc;
}

/* ---------------------------------------------------------------------------
 * Bit-reversible kick-drift-kick with fixed-point state (the integer-state
 * idea of Rein and Tamayo's JANUS integrator, 2018, applied to the leapfrog
 * of Section IV.B's Move_bodies).  Positions and velocities are integers in
 * units of 2^-sx and 2^-sv.  With the force a(x) of the decoded positions
 * (decode: x = X * 2^-sx, exact in FP64 for |X| < 2^53):
 *   kick:  V += round(kick_scale * a),  kick_scale = h G 2^sv
 *   drift: X += round((double)V * drift_scale),  drift_scale = dt 2^(sx-sv)
 * round() is round-half-to-even of the FP64 product.  Every increment depends
 * only on the state it does not change, so subtracting the same integers
 * undoes a step exactly.  One force evaluation per step; the oracle uses its
 * FP64 force (G = 1 in the evaluation, G in kick_scale).
 * state: int64 [n][8] = (X, Y, Z, 0, VX, VY, VZ, 0).
 * ------------------------------------------------------------------------- */
static void janus_decode(int64_t n, const int64_t *st, double inv_sx, double *x)
{
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k)
            x[3 * i + k] = (double)st[8 * i + k] * inv_sx;
}

static void janus_kick(int64_t n, int64_t *st, const double *a, double kick_scale, int64_t sign)
{
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k)
            st[8 * i + 4 + k] += sign * (int64_t)nearbyint(kick_scale * a[3 * i + k]);
}

static void janus_drift(int64_t n, int64_t *st, double drift_scale, int64_t sign)
{
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k)
            st[8 * i + k] += sign * (int64_t)nearbyint((double)st[8 * i + 4 + k] * drift_scale);
}

/* direction +1: nsteps forward; -1: nsteps backward (exact inverse). */
int oracle_janus_run(int64_t n, int64_t *state, const double *m, double G, double eps, double dt,
                     int32_t nsteps, int32_t sx, int32_t sv, int32_t direction)
{
    if (n < 1 || nsteps < 0 || (direction != 1 && direction != -1))
        return -1;
    double *x = (double *)malloc((size_t)n * 3 * sizeof(double));
    double *a = (double *)malloc((size_t)n * 3 * sizeof(double));
    if (!x || !a) {
        free(x);
        free(a);
        return -1;
    }
    const double inv_sx = ldexp(1.0, -sx);
    const double kick_scale = 0.5 * dt * G * ldexp(1.0, sv);
    const double drift_scale = dt * ldexp(1.0, sx - sv);
    janus_decode(n, state, inv_sx, x);
    oracle_accel(n, x, m, 1.0, eps, n, NULL, a, NULL);
    for (int32_t s = 0; s < nsteps; ++s) {
        if (direction > 0) {
            janus_kick(n, state, a, kick_scale, 1);
            janus_drift(n, state, drift_scale, 1);
            janus_decode(n, state, inv_sx, x);
            oracle_accel(n, x, m, 1.0, eps, n, NULL, a, NULL);
            janus_kick(n, state, a, kick_scale, 1);
        } else {
            janus_kick(n, state, a, kick_scale, -1);
            janus_drift(n, state, drift_scale, -1);
            janus_decode(n, state, inv_sx, x);
            oracle_accel(n, x, m, 1.0, eps, n, NULL, a, NULL);
            janus_kick(n, state, a, kick_scale, -1);
        }
    }
    free(x);
    free(a);
    return 0;
}
