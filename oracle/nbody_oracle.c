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
 *                    L = sum_i |x_i(T) - y_i|^2, storing every state.
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
