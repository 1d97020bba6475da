/*
 * oracle.c -- plain, slow, FP64 CPU reference of the Trotter-Suzuki spin propagator
 * of Dente, Bederian, Zangara and Pastawski, "GPU accelerated Trotter-Suzuki solver
 * for quantum spin dynamics" (arXiv:1305.0036).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or calls
 * this file.  Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no source with the GPU path.
 *
 * What it computes, in the paper's order and notation:
 *   - H = sum_j sum_a h^a_j S^a_j + sum_(j,k) sum_a J^a_jk S^a_j S^a_k     (Sec. 2, Eq. 1)
 *     split by axis into K = 3 parts H_a = sum_j h^a_j S^a_j + sum_(j,k) J^a_jk S^a_j S^a_k
 *     (Sec. 2: field and coupling terms of one axis are rotated together).
 *   - The state is the 2^N coefficient vector in the Ising basis (Sec. 2, Eq. 2).  Spin j
 *     is bit j of the basis index, counted from the right (Sec. 3.2 footnote); a set bit
 *     is spin up, s_j = +1/2 (Sec. 3.3, F-set example).
 *   - U1(t) = exp(-itH_1)...exp(-itH_K) (Eq. U1).  With H_1 = H_x, H_2 = H_y, H_3 = H_z the
 *     z part acts first on the state.
 *   - U2(t) = U1^dagger(-t/2) U1(t/2);  U4(t) = U2(at)U2(at)U2((1-4a)t)U2(at)U2(at),
 *     a = 1/(4 - 4^(1/3))  (Sec. 2, second and fourth order products).
 *   - exp(-itH_a) for a = x, y is evaluated as V_a exp(-it D_a) V_a^dagger, where V_a is a
 *     product of one 2x2 rotation per spin with V^dagger S^a V = S^z, and D_a(b) is the
 *     diagonal of H_a with S^a replaced by S^z (Sec. 2, Eqs. Single Spin Rotation and
 *     Two-Spin-Operators).  The z part is the diagonal phase exp(-it D_z(b))
 *     (Sec. 2, Eq. ZZ-Phases, evolved with the sign of exp(-itH)).
 *   - V_a here is the oracle's own choice: the eigenvector matrix of S^a with columns
 *     ordered as diag(-1/2, +1/2).  exp(-itH_a) does not depend on that choice.
 *
 * Plain loops only: one spin at a time, one pair at a time, no tiling, no fusion, no
 * tables and no merging of consecutive phases.  OpenMP is used over pairs and basis
 * indices only.  All arithmetic is double precision.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

enum { AX_X = 0, AX_Y = 1, AX_Z = 2 };
enum {
    OBS_NORM = 0, OBS_SX = 1, OBS_SY = 2, OBS_SZ = 3, OBS_SZSZ = 4,
    OBS_MZ = 5, OBS_ENERGY = 6, OBS_OVERLAP_SZ = 7
};

/* s_j(b): +1/2 when bit j of b is set (spin up), -1/2 otherwise. */
static inline double spin_z(uint64_t b, int j) { return ((b >> j) & 1u) ? 0.5 : -0.5; }

/* ---------------------------------------------------------------- one-spin matrices */

/* S^x, S^y, S^z in the one-spin basis ordered (down, up). */
static void spin_matrix(int axis, cplx S[2][2])
{
    memset(S, 0, 4 * sizeof(cplx));
    if (axis == AX_X) { S[0][1] = 0.5; S[1][0] = 0.5; }
    else if (axis == AX_Y) { S[0][1] = 0.5 * I; S[1][0] = -0.5 * I; }
    else { S[0][0] = -0.5; S[1][1] = 0.5; }
}

/* V_a: columns are the eigenvectors of S^a for eigenvalues -1/2 and +1/2. */
static void rot_matrix(int axis, cplx V[2][2])
{
    const double r = 1.0 / sqrt(2.0);
    if (axis == AX_X) {          /* (1,-1)/sqrt2 -> -1/2 ; (1,1)/sqrt2 -> +1/2 */
        V[0][0] = r;  V[0][1] = r;
        V[1][0] = -r; V[1][1] = r;
    } else {                     /* (-i,1)/sqrt2 -> -1/2 ; (i,1)/sqrt2 -> +1/2 */
        V[0][0] = -I * r; V[0][1] = I * r;
        V[1][0] = r;      V[1][1] = r;
    }
}

static void dagger(const cplx A[2][2], cplx B[2][2])
{
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) B[r][c] = conj(A[c][r]);
}

/* Largest |V^dagger S^a V - S^z| entry over a = x, y, and |V^dagger V - 1|. */
double orc_selfcheck(void)
{
    double worst = 0.0;
    cplx Sz[2][2];
    spin_matrix(AX_Z, Sz);
    for (int axis = AX_X; axis <= AX_Y; ++axis) {
        cplx S[2][2], V[2][2], Vd[2][2], T[2][2], R[2][2];
        spin_matrix(axis, S);
        rot_matrix(axis, V);
        dagger(V, Vd);
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 2; ++c) {
                T[r][c] = 0;
                for (int k = 0; k < 2; ++k) T[r][c] += S[r][k] * V[k][c];
            }
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 2; ++c) {
                R[r][c] = 0;
                for (int k = 0; k < 2; ++k) R[r][c] += Vd[r][k] * T[k][c];
                double d = cabs(R[r][c] - Sz[r][c]);
                if (d > worst) worst = d;
                cplx u = 0;
                for (int k = 0; k < 2; ++k) u += Vd[r][k] * V[k][c];
                d = cabs(u - (r == c ? 1.0 : 0.0));
                if (d > worst) worst = d;
            }
    }
    return worst;
}

/* ------------------------------------------------------------------------- energy */

/* D_a(b) = sum_j h^a_j s_j(b) + sum_bonds J^a s_i(b) s_j(b), terms in listed order. */
double orc_energy(int n, int nb, const int *bi, const int *bj, const double *J,
                  const double *h, int axis, uint64_t b)
{
    double e = 0.0;
    for (int j = 0; j < n; ++j) e += h[3 * j + axis] * spin_z(b, j);
    for (int k = 0; k < nb; ++k) e += J[3 * k + axis] * spin_z(b, bi[k]) * spin_z(b, bj[k]);
    return e;
}

void orc_energies(int n, int nb, const int *bi, const int *bj, const double *J,
                  const double *h, int axis, const uint64_t *bs, int64_t count, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < count; ++k) out[k] = orc_energy(n, nb, bi, bj, J, h, axis, bs[k]);
}

/* ------------------------------------------------------------------ elementary ops */

/* Apply a 2x2 matrix U to spin q: every pair (b, b + 2^q) with bit q of b clear. */
void orc_apply_1spin(int n, cplx *psi, int q, const cplx U[2][2])
{
    const int64_t half = (int64_t)1 << (n - 1);
    const uint64_t m = (uint64_t)1 << q;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < half; ++p) {
        uint64_t lo = (uint64_t)p & (m - 1);
        uint64_t b = (((uint64_t)p - lo) << 1) | lo;
        cplx c0 = psi[b], c1 = psi[b | m];
        psi[b] = U[0][0] * c0 + U[0][1] * c1;
        psi[b | m] = U[1][0] * c0 + U[1][1] * c1;
    }
}

/* c_b <- c_b exp(-i tau D_a(b)). */
static void apply_phase(int n, int nb, const int *bi, const int *bj, const double *J,
                        const double *h, int axis, double tau, cplx *psi)
{
    const int64_t dim = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < dim; ++b) {
        double phi = tau * orc_energy(n, nb, bi, bj, J, h, axis, (uint64_t)b);
        psi[b] *= cos(phi) - I * sin(phi);
    }
}

static void rotate_all(int n, cplx *psi, int axis, int adjoint)
{
    cplx V[2][2], Vd[2][2];
    rot_matrix(axis, V);
    dagger(V, Vd);
    for (int q = 0; q < n; ++q) orc_apply_1spin(n, psi, q, adjoint ? Vd : V);
}

/* One partial evolution exp(-i tau H_a). */
void orc_substep(int n, int nb, const int *bi, const int *bj, const double *J,
                 const double *h, int axis, double tau, cplx *psi)
{
    if (axis == AX_Z) {
        apply_phase(n, nb, bi, bj, J, h, AX_Z, tau, psi);
        return;
    }
    rotate_all(n, psi, axis, 1);                 /* V^dagger: S^a -> S^z frame */
    apply_phase(n, nb, bi, bj, J, h, axis, tau, psi);
    rotate_all(n, psi, axis, 0);                 /* back to the Ising basis    */
}

/* ------------------------------------------------------------------------ schedule */

double orc_suzuki_a(void) { return 1.0 / (4.0 - cbrt(4.0)); }

/*
 * Sub-steps (axis, tau) of one step of the given order, in the order they act on the
 * state.  Returns the count (3, 6 or 30), or -1 for an unknown order.
 *   U1(t): z(t), y(t), x(t).
 *   U2(t) = U1^dagger(-t/2) U1(t/2): U1(t/2) acts first [z, y, x at t/2], then
 *           U1^dagger(-t/2) = exp(-i t/2 H_z) exp(-i t/2 H_y) exp(-i t/2 H_x) acts,
 *           i.e. x, y, z at t/2.
 *   U4(t): U2(at) U2(at) U2((1-4a)t) U2(at) U2(at).
 */
int orc_step_schedule(int order, double dt, int *axes, double *taus)
{
    int k = 0;
    if (order == 1) {
        axes[k] = AX_Z; taus[k++] = dt;
        axes[k] = AX_Y; taus[k++] = dt;
        axes[k] = AX_X; taus[k++] = dt;
        return k;
    }
    if (order == 2) {
        const double h2 = 0.5 * dt;
        axes[k] = AX_Z; taus[k++] = h2;
        axes[k] = AX_Y; taus[k++] = h2;
        axes[k] = AX_X; taus[k++] = h2;
        axes[k] = AX_X; taus[k++] = h2;
        axes[k] = AX_Y; taus[k++] = h2;
        axes[k] = AX_Z; taus[k++] = h2;
        return k;
    }
    if (order == 4) {
        const double a = orc_suzuki_a();
        const double ts[5] = { a * dt, a * dt, (1.0 - 4.0 * a) * dt, a * dt, a * dt };
        for (int u = 0; u < 5; ++u) {
            k += orc_step_schedule(2, ts[u], axes + k, taus + k);
        }
        return k;
    }
    return -1;
}

int orc_evolve(int n, int nb, const int *bi, const int *bj, const double *J,
               const double *h, cplx *psi, double dt, int64_t nsteps, int order)
{
    int axes[32];
    double taus[32];
    int ns = orc_step_schedule(order, dt, axes, taus);
    if (ns < 0) return -1;
    for (int64_t s = 0; s < nsteps; ++s)
        for (int k = 0; k < ns; ++k) orc_substep(n, nb, bi, bj, J, h, axes[k], taus[k], psi);
    return 0;
}

/* ---------------------------------------------------------------------- observables */

/* out = O psi for the Hermitian observables; out must not alias psi. */
static void apply_spin_op(int n, int axis, int j, const cplx *psi, cplx *out)
{
    const int64_t dim = (int64_t)1 << n;
    const uint64_t m = (uint64_t)1 << j;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < dim; ++b) {
        uint64_t ub = (uint64_t)b;
        if (axis == AX_Z) {
            out[b] = spin_z(ub, j) * psi[b];
        } else if (axis == AX_X) {
            out[b] = 0.5 * psi[ub ^ m];
        } else {
            /* (S^y psi)_down = (i/2) c_up ; (S^y psi)_up = (-i/2) c_down */
            out[b] = (((ub >> j) & 1u) ? -0.5 * I : 0.5 * I) * psi[ub ^ m];
        }
    }
}

int orc_apply_obs(int n, int nb, const int *bi, const int *bj, const double *J,
                  const double *h, int kind, int i, int j, const cplx *psi, cplx *out)
{
    const int64_t dim = (int64_t)1 << n;
    switch (kind) {
    case OBS_NORM:
        memcpy(out, psi, (size_t)dim * sizeof(cplx));
        return 0;
    case OBS_SX: apply_spin_op(n, AX_X, i, psi, out); return 0;
    case OBS_SY: apply_spin_op(n, AX_Y, i, psi, out); return 0;
    case OBS_SZ: apply_spin_op(n, AX_Z, i, psi, out); return 0;
    case OBS_SZSZ:
#pragma omp parallel for schedule(static)
        for (int64_t b = 0; b < dim; ++b)
            out[b] = spin_z((uint64_t)b, i) * spin_z((uint64_t)b, j) * psi[b];
        return 0;
    case OBS_MZ:
#pragma omp parallel for schedule(static)
        for (int64_t b = 0; b < dim; ++b) {
            double m = 0.0;
            for (int q = 0; q < n; ++q) m += spin_z((uint64_t)b, q);
            out[b] = m * psi[b];
        }
        return 0;
    case OBS_ENERGY: {
        cplx *t1 = malloc((size_t)dim * sizeof(cplx));
        cplx *t2 = malloc((size_t)dim * sizeof(cplx));
        if (!t1 || !t2) { free(t1); free(t2); return -2; }
        memset(out, 0, (size_t)dim * sizeof(cplx));
        for (int axis = AX_X; axis <= AX_Z; ++axis) {
            for (int q = 0; q < n; ++q) {
                double hq = h[3 * q + axis];
                if (hq == 0.0) continue;
                apply_spin_op(n, axis, q, psi, t1);
                for (int64_t b = 0; b < dim; ++b) out[b] += hq * t1[b];
            }
            for (int k = 0; k < nb; ++k) {
                double jk = J[3 * k + axis];
                if (jk == 0.0) continue;
                apply_spin_op(n, axis, bj[k], psi, t1);
                apply_spin_op(n, axis, bi[k], t1, t2);
                for (int64_t b = 0; b < dim; ++b) out[b] += jk * t2[b];
            }
        }
        free(t1);
        free(t2);
        return 0;
    }
    default:
        return -1;
    }
}

/* Neumaier-compensated sum of <a|b> = sum conj(a_b) b_b, real and imaginary parts. */
static void inner(int64_t dim, const cplx *a, const cplx *b, double out[2])
{
    double sr = 0.0, cr = 0.0, si = 0.0, ci = 0.0;
    for (int64_t k = 0; k < dim; ++k) {
        cplx z = conj(a[k]) * b[k];
        double x = creal(z), t = sr + x;
        cr += (fabs(sr) >= fabs(x)) ? (sr - t) + x : (x - t) + sr;
        sr = t;
        x = cimag(z);
        t = si + x;
        ci += (fabs(si) >= fabs(x)) ? (si - t) + x : (x - t) + si;
        si = t;
    }
    out[0] = sr + cr;
    out[1] = si + ci;
}

/*
 * <psi|O|psi> (real, out[1] = 0 up to rounding) or, for OBS_OVERLAP_SZ, the complex
 * <other|S^z_i|psi>.  Returns 0, or -1 for an unknown kind.
 */
int orc_expect(int n, int nb, const int *bi, const int *bj, const double *J,
               const double *h, const cplx *psi, int kind, int i, int j,
               const cplx *other, double out[2])
{
    const int64_t dim = (int64_t)1 << n;
    cplx *t = malloc((size_t)dim * sizeof(cplx));
    if (!t) return -2;
    int rc;
    if (kind == OBS_OVERLAP_SZ) {
        apply_spin_op(n, AX_Z, i, psi, t);
        inner(dim, other, t, out);
        rc = 0;
    } else {
        rc = orc_apply_obs(n, nb, bi, bj, J, h, kind, i, j, psi, t);
        if (rc == 0) inner(dim, psi, t, out);
    }
    free(t);
    return rc;
}

/* ------------------------------------------------------------- forward-mode gradient */

/*
 * Derivative of L = <psi(T)|O|psi(T)> with respect to every coupling J^a of every listed
 * bond and every field h^a_j, by forward-mode tangents: for a parameter theta that
 * enters D_a with weight f(b) (s_j(b) for h^a_j, s_i(b)s_j(b) for J^a_ij), every partial
 * evolution G = V exp(-i tau D_a) V^dagger of that axis has
 *     dG/dtheta = V (-i tau f) exp(-i tau D_a) V^dagger,
 * so the pair (psi, dpsi) advances as dpsi <- G dpsi + (dG/dtheta) psi, psi <- G psi.
 * At the end dL/dtheta = 2 Re <O psi | dpsi>.  One tangent run per parameter.
 * For the energy O = H of Eq. 1 the observable itself depends on theta, and the product
 * rule adds <psi(T)| dH/dtheta |psi(T)>: <S^a_j> for h^a_j, <S^a_i S^a_j> for J^a_ij.
 * grad_bonds is [nb][3] and grad_fields is [n][3] (x, y, z).
 */
int orc_grad_forward(int n, int nb, const int *bi, const int *bj, const double *J,
                     const double *h, const cplx *psi0, double dt, int64_t nsteps,
                     int order, int kind, int oi, int oj, double *loss,
                     double *grad_bonds, double *grad_fields)
{
    if (kind == OBS_NORM || kind == OBS_OVERLAP_SZ) return -1;
    int axes[32];
    double taus[32];
    int ns = orc_step_schedule(order, dt, axes, taus);
    if (ns < 0) return -1;
    const int64_t dim = (int64_t)1 << n;
    cplx *psi = malloc((size_t)dim * sizeof(cplx));
    cplx *dpsi = malloc((size_t)dim * sizeof(cplx));
    cplx *opsi = malloc((size_t)dim * sizeof(cplx));
    cplx *t1 = malloc((size_t)dim * sizeof(cplx));
    cplx *t2 = malloc((size_t)dim * sizeof(cplx));
    if (!psi || !dpsi || !opsi || !t1 || !t2) {
        free(psi); free(dpsi); free(opsi); free(t1); free(t2);
        return -2;
    }

    const int nparam = 3 * nb + 3 * n;
    for (int p = 0; p < nparam; ++p) {
        int is_bond = p < 3 * nb;
        int idx = is_bond ? p / 3 : (p - 3 * nb) / 3;
        int paxis = is_bond ? p % 3 : (p - 3 * nb) % 3;
        memcpy(psi, psi0, (size_t)dim * sizeof(cplx));
        memset(dpsi, 0, (size_t)dim * sizeof(cplx));
        for (int64_t s = 0; s < nsteps; ++s) {
            for (int k = 0; k < ns; ++k) {
                int axis = axes[k];
                double tau = taus[k];
                if (axis != AX_Z) { rotate_all(n, psi, axis, 1); rotate_all(n, dpsi, axis, 1); }
#pragma omp parallel for schedule(static)
                for (int64_t b = 0; b < dim; ++b) {
                    uint64_t ub = (uint64_t)b;
                    double phi = tau * orc_energy(n, nb, bi, bj, J, h, axis, ub);
                    cplx ph = cos(phi) - I * sin(phi);
                    cplx d = dpsi[b];
                    if (axis == paxis) {
                        double f = is_bond ? spin_z(ub, bi[idx]) * spin_z(ub, bj[idx])
                                           : spin_z(ub, idx);
                        d += -I * tau * f * psi[b];
                    }
                    dpsi[b] = ph * d;
                    psi[b] = ph * psi[b];
                }
                if (axis != AX_Z) { rotate_all(n, psi, axis, 0); rotate_all(n, dpsi, axis, 0); }
            }
        }
        orc_apply_obs(n, nb, bi, bj, J, h, kind, oi, oj, psi, opsi);
        double ip[2];
        inner(dim, opsi, dpsi, ip);
        double g = 2.0 * ip[0];
        if (kind == OBS_ENERGY) {
            /* explicit term: the spin operator (or product) that theta multiplies in H */
            if (is_bond) {
                apply_spin_op(n, paxis, bj[idx], psi, t1);
                apply_spin_op(n, paxis, bi[idx], t1, t2);
            } else {
                apply_spin_op(n, paxis, idx, psi, t2);
            }
            inner(dim, psi, t2, ip);
            g += ip[0];
        }
        if (is_bond) grad_bonds[3 * idx + paxis] = g;
        else grad_fields[3 * idx + paxis] = g;
        if (p == 0) {
            inner(dim, psi, opsi, ip);
            *loss = ip[0];
        }
    }
    if (nparam == 0) {
        memcpy(psi, psi0, (size_t)dim * sizeof(cplx));
        orc_evolve(n, nb, bi, bj, J, h, psi, dt, nsteps, order);
        orc_apply_obs(n, nb, bi, bj, J, h, kind, oi, oj, psi, opsi);
        double ip[2];
        inner(dim, psi, opsi, ip);
        *loss = ip[0];
    }
    free(psi);
    free(dpsi);
    free(opsi);
    free(t1);
    free(t2);
    return 0;
}
