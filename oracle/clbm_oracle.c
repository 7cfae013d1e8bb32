/*
 * clbm_oracle.c -- TEST INFRASTRUCTURE ONLY (the oracle).
 *
 * A plain, slow, FP64 CPU reference of the D2Q9 cascaded lattice Boltzmann
 * method (CLBM) with the consistent forcing scheme of Fei & Luo,
 * "Consistent forcing scheme in the cascaded lattice Boltzmann method".
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no code, header, table or
 * helper with the GPU library, and the GPU library never loads it.
 *
 * How it is written:
 *   - the transformation matrix M (Eq. 5), the shift matrix N(u) (Eq. 6)
 *     and the inverses M^-1 and N^-1(u) (Appendix) are typed in as printed
 *     and applied as dense 9x9 matrix-vector products;
 *   - one time step takes the paper's steps in its order: density and
 *     velocity (Eqs. 11 and 15), raw moments T = M f and central moments
 *     T~ = N T (Eq. 4), relaxation with the force moments (Eq. 12, first
 *     line), back-transform f* = M^-1 N^-1 T~* (Eq. 9), then streaming
 *     f_i(x + e_i) = f_i*(x) in push form (Eq. 10), with half-way
 *     bounce-back where x + e_i lies beyond a wall (Sec. IV A);
 *   - no blocking, fusion or reordering beyond that.
 *
 * Readings of the paper taken here (each is listed with its reason in the
 * design notes of the repository):
 *   - Eq. (14) prints the third-order slots of C as (cs^2 Fx, cs^2 Fy) in
 *     the (k~21, k~12) positions.  Deriving them from Eq. (13) with the
 *     equilibrium of Eq. (8) gives k~21 -> cs^2 Fy and k~12 -> cs^2 Fx,
 *     and only that order is covariant under x -> -x.  C is therefore
 *     [0, Fx, Fy, 0, 0, 0, cs^2 Fy, cs^2 Fx, 0].
 *   - The second line of Eq. (12) lacks the (I - S) factor; the first line
 *     is used.
 *   - The velocity in N(u) and N^-1(u) is the forced velocity of Eq. (15).
 *   - The weights w_i (Remark 3) are the rest equilibrium f_i^eq(rho=1,u=0):
 *     4/9, 1/9 (x4), 1/36 (x4).
 *   - The initial state is the pre-collision f whose central moments are
 *     [rho, -Fx/2, -Fy/2, 2 rho cs^2, 0, 0, 0, 0, rho cs^4]: its Eq. (15)
 *     velocity is exactly the requested u.  The paper does not state it.
 *
 * Parity pins (tests that tie this file to something other than itself) are
 * listed in the test suite; none of the functions here is "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 9

/* Eq. (1): D2Q9 velocities, c = dx/dt = 1. */
static const int EX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
/* Direction opposite to i (e_opp = -e_i), used by bounce-back. */
static const int OPP[Q] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
/* Sec. II A: lattice sound speed squared. */
static const double CS2 = 1.0 / 3.0;

/* Eq. (5): T = M f with T = [k00,k10,k01,k20+k02,k20-k02,k11,k21,k12,k22]. */
static const double MMAT[Q][Q] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 1, 1, 1, 1, 2, 2, 2, 2},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1},
    {0, 0, 0, 0, 0, 1, 1, -1, -1},
    {0, 0, 0, 0, 0, 1, -1, -1, 1},
    {0, 0, 0, 0, 0, 1, 1, 1, 1},
};

/* Appendix: M^-1 as printed. */
static const double MINV[Q][Q] = {
    {1, 0, 0, -1, 0, 0, 0, 0, 1},
    {0, 0.5, 0, 0.25, 0.25, 0, 0, -0.5, -0.5},
    {0, 0, 0.5, 0.25, -0.25, 0, -0.5, 0, -0.5},
    {0, -0.5, 0, 0.25, 0.25, 0, 0, 0.5, -0.5},
    {0, 0, -0.5, 0.25, -0.25, 0, 0.5, 0, -0.5},
    {0, 0, 0, 0, 0, 0.25, 0.25, 0.25, 0.25},
    {0, 0, 0, 0, 0, -0.25, 0.25, -0.25, 0.25},
    {0, 0, 0, 0, 0, 0.25, -0.25, -0.25, 0.25},
    {0, 0, 0, 0, 0, -0.25, -0.25, 0.25, 0.25},
};

/* Eq. (6): the shift matrix N(u), T~ = N T, entry by entry as printed. */
static void shift_matrix(double ux, double uy, double N[Q][Q])
{
    memset(N, 0, sizeof(double) * Q * Q);
    const double ux2 = ux * ux, uy2 = uy * uy;
    N[0][0] = 1.0;

    N[1][0] = -ux;
    N[1][1] = 1.0;

    N[2][0] = -uy;
    N[2][2] = 1.0;

    N[3][0] = ux2 + uy2;
    N[3][1] = -2.0 * ux;
    N[3][2] = -2.0 * uy;
    N[3][3] = 1.0;

    N[4][0] = ux2 - uy2;
    N[4][1] = -2.0 * ux;
    N[4][2] = 2.0 * uy;
    N[4][4] = 1.0;

    N[5][0] = ux * uy;
    N[5][1] = -uy;
    N[5][2] = -ux;
    N[5][5] = 1.0;

    N[6][0] = -ux2 * uy;
    N[6][1] = 2.0 * ux * uy;
    N[6][2] = ux2;
    N[6][3] = -uy / 2.0;
    N[6][4] = -uy / 2.0;
    N[6][5] = -2.0 * ux;
    N[6][6] = 1.0;

    N[7][0] = -uy2 * ux;
    N[7][1] = uy2;
    N[7][2] = 2.0 * ux * uy;
    N[7][3] = -ux / 2.0;
    N[7][4] = ux / 2.0;
    N[7][5] = -2.0 * uy;
    N[7][7] = 1.0;

    N[8][0] = ux2 * uy2;
    N[8][1] = -2.0 * ux * uy2;
    N[8][2] = -2.0 * uy * ux2;
    N[8][3] = ux2 / 2.0 + uy2 / 2.0;
    N[8][4] = uy2 / 2.0 - ux2 / 2.0;
    N[8][5] = 4.0 * ux * uy;
    N[8][6] = -2.0 * uy;
    N[8][7] = -2.0 * ux;
    N[8][8] = 1.0;
}

/* Appendix: N^-1(u), T = N^-1 T~, entry by entry as printed. */
static void shift_matrix_inverse(double ux, double uy, double NI[Q][Q])
{
    memset(NI, 0, sizeof(double) * Q * Q);
    const double ux2 = ux * ux, uy2 = uy * uy;
    NI[0][0] = 1.0;

    NI[1][0] = ux;
    NI[1][1] = 1.0;

    NI[2][0] = uy;
    NI[2][2] = 1.0;

    NI[3][0] = ux2 + uy2;
    NI[3][1] = 2.0 * ux;
    NI[3][2] = 2.0 * uy;
    NI[3][3] = 1.0;

    NI[4][0] = ux2 - uy2;
    NI[4][1] = 2.0 * ux;
    NI[4][2] = -2.0 * uy;
    NI[4][4] = 1.0;

    NI[5][0] = ux * uy;
    NI[5][1] = uy;
    NI[5][2] = ux;
    NI[5][5] = 1.0;

    NI[6][0] = ux2 * uy;
    NI[6][1] = 2.0 * ux * uy;
    NI[6][2] = ux2;
    NI[6][3] = uy / 2.0;
    NI[6][4] = uy / 2.0;
    NI[6][5] = 2.0 * ux;
    NI[6][6] = 1.0;

    NI[7][0] = uy2 * ux;
    NI[7][1] = uy2;
    NI[7][2] = 2.0 * ux * uy;
    NI[7][3] = ux / 2.0;
    NI[7][4] = -ux / 2.0;
    NI[7][5] = 2.0 * uy;
    NI[7][7] = 1.0;

    NI[8][0] = ux2 * uy2;
    NI[8][1] = 2.0 * ux * uy2;
    NI[8][2] = 2.0 * uy * ux2;
    NI[8][3] = ux2 / 2.0 + uy2 / 2.0;
    NI[8][4] = uy2 / 2.0 - ux2 / 2.0;
    NI[8][5] = 4.0 * ux * uy;
    NI[8][6] = 2.0 * uy;
    NI[8][7] = 2.0 * ux;
    NI[8][8] = 1.0;
}

/* y = A x for a 9x9 matrix, summed in index order. */
static void matvec(const double A[Q][Q], const double x[Q], double y[Q])
{
    for (int r = 0; r < Q; ++r) {
        double acc = 0.0;
        for (int c = 0; c < Q; ++c) acc += A[r][c] * x[c];
        y[r] = acc;
    }
}

/* Rest weights w_i = f_i^eq(rho = 1, u = 0) (Remark 3 uses them). */
static const double W[Q] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                            1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

/* Forcing schemes the oracle knows. */
enum {
    ORACLE_SCHEME_CONSISTENT = 0, /* Eq. (12) with C from Eq. (14)       */
    ORACLE_SCHEME_GUO_LBL = 1,    /* Eq. (21): (1 - s2/2) N M R_G        */
    ORACLE_SCHEME_PREMNATH = 2    /* Eqs. (17)-(19), Sec. III A          */
};

/*
 * Sec. III A (Premnath et al.): the central moments of the force's change
 * of the distribution, with the higher-order ones dropped (Eq. 19):
 * C_P = [0, Fx, Fy, 0, 0, 0, 0, 0, 0].  The paper cites the discrete
 * change Delta f_i without printing it; it is read here as the discrete
 * distribution whose central moments about u are exactly C_P, i.e.
 * Delta f = M^-1 N^-1(u) C_P.  That reading gives the leading term of
 * Eq. (20), Delta f_0 = -2 F.u + O(u^3), and makes the scheme coincide
 * with Eq. (12) at s3 = 2 (Remark 6).
 */
static void premnath_moments(double Fx, double Fy, double CP[Q])
{
    memset(CP, 0, sizeof(double) * Q);
    CP[1] = Fx;
    CP[2] = Fy;
}

/* Delta f_i of Sec. III A at velocity u (the reading above). */
static void premnath_delta_f(double Fx, double Fy, double ux, double uy, double df[Q])
{
    double CP[Q], NI[Q][Q], T[Q];
    premnath_moments(Fx, Fy, CP);
    shift_matrix_inverse(ux, uy, NI);
    matvec(NI, CP, T);
    matvec(MINV, T, df);
}

/* Guo's forcing term R_Gi (Remark 3) at velocity u. */
static void guo_force_term(double Fx, double Fy, double ux, double uy, double R[Q])
{
    for (int i = 0; i < Q; ++i) {
        const double eu = EX[i] * ux + EY[i] * uy;
        const double ax = (EX[i] - ux) / CS2 + eu * EX[i] / (CS2 * CS2);
        const double ay = (EY[i] - uy) / CS2 + eu * EY[i] / (CS2 * CS2);
        R[i] = W[i] * (ax * Fx + ay * Fy);
    }
}

/*
 * One collision at one node.
 *   f[9]      pre-collision populations
 *   Fx, Fy    force density at the node
 *   s6        {s0, s1, sb, s2, s3, s4}; S = diag(s0,s1,s1,sb,s2,s2,s3,s3,s4)
 *   scheme    ORACLE_SCHEME_*
 *   shift     1: N(u) as printed (the CLBM).  0: N replaced by the identity
 *             (Remark 2): the relaxation acts on raw moments, with the
 *             equilibrium and force vectors carried to raw moments by
 *             N^-1(u).
 *   fout[9]   post-collision populations f*
 */
static void collide(const double f[Q], double Fx, double Fy, const double s6[6],
                    int scheme, int shift, double fout[Q])
{
    /* Eq. (11) and Eq. (15). */
    double rho = 0.0, jx = 0.0, jy = 0.0;
    for (int i = 0; i < Q; ++i) {
        rho += f[i];
        jx += f[i] * EX[i];
        jy += f[i] * EY[i];
    }
    const double ux = (jx + 0.5 * Fx) / rho;
    const double uy = (jy + 0.5 * Fy) / rho;

    /* S = diag(s0, s1, s1, sb, s2, s2, s3, s3, s4). */
    const double S[Q] = {s6[0], s6[1], s6[1], s6[2], s6[3], s6[3], s6[4], s6[4], s6[5]};

    double N[Q][Q], NI[Q][Q];
    shift_matrix(ux, uy, N);
    shift_matrix_inverse(ux, uy, NI);

    /* Eq. (4): raw moments, then central moments. */
    double T[Q], Tt[Q];
    matvec(MMAT, f, T);
    if (shift)
        matvec(N, T, Tt);
    else
        memcpy(Tt, T, sizeof T);

    /* Eq. (8): equilibrium central moments. */
    double Teq[Q] = {rho, 0, 0, 2.0 * rho * CS2, 0, 0, 0, 0, rho * CS2 * CS2};

    /* Eq. (14), slots 6 and 7 read as (cs^2 Fy, cs^2 Fx). */
    double C[Q] = {0, Fx, Fy, 0, 0, 0, CS2 * Fy, CS2 * Fx, 0};

    /* Eq. (21): central moments of Guo's term, N M R_G. */
    double CG[Q];
    if (scheme == ORACLE_SCHEME_GUO_LBL) {
        double R[Q], MR[Q];
        guo_force_term(Fx, Fy, ux, uy, R);
        matvec(MMAT, R, MR);
        matvec(N, MR, CG);
    }

    /* Eq. (19): the force's central moments in the scheme of Sec. III A. */
    double CP[Q];
    premnath_moments(Fx, Fy, CP);

    if (!shift) {
        /* Remark 2: with N = I the same vectors are expressed as raw moments. */
        double tmp[Q];
        matvec(NI, Teq, tmp);
        memcpy(Teq, tmp, sizeof tmp);
        matvec(NI, C, tmp);
        memcpy(C, tmp, sizeof tmp);
        if (scheme == ORACLE_SCHEME_GUO_LBL) {
            matvec(NI, CG, tmp);
            memcpy(CG, tmp, sizeof tmp);
        }
        matvec(NI, CP, tmp);
        memcpy(CP, tmp, sizeof tmp);
    }

    /* Eq. (12) first line (consistent), Eq. (21) (Lycett-Brown & Luo), or
     * Eq. (17) (Premnath et al.: relaxation toward T~eq - C_P/2). */
    double Ts[Q];
    for (int k = 0; k < Q; ++k) {
        if (scheme == ORACLE_SCHEME_PREMNATH) {
            Ts[k] = (1.0 - S[k]) * Tt[k] + S[k] * (Teq[k] - CP[k] / 2.0);
            continue;
        }
        Ts[k] = (1.0 - S[k]) * Tt[k] + S[k] * Teq[k];
        if (scheme == ORACLE_SCHEME_GUO_LBL)
            Ts[k] += (1.0 - s6[3] / 2.0) * CG[k];
        else
            Ts[k] += (1.0 - S[k] / 2.0) * C[k];
    }

    /* Eq. (9): f* = M^-1 N^-1 T~*. */
    double Tr[Q];
    if (shift)
        matvec(NI, Ts, Tr);
    else
        memcpy(Tr, Ts, sizeof Ts);
    matvec(MINV, Tr, fout);

    /* Eq. (18): the scheme of Sec. III A adds the discrete change Delta f
     * (CP already holds raw moments when N = I). */
    if (scheme == ORACLE_SCHEME_PREMNATH) {
        double df[Q];
        if (shift) {
            premnath_delta_f(Fx, Fy, ux, uy, df);
        } else {
            matvec(MINV, CP, df);
        }
        for (int i = 0; i < Q; ++i) fout[i] += df[i];
    }
}

/* ----------------------------------------------------------------------- */
/* Exported entry points.  Lattice arrays are [9][ny][nx], x fastest.       */
/* ----------------------------------------------------------------------- */

void oracle_matrix_M(double *out)
{
    memcpy(out, MMAT, sizeof MMAT);
}

void oracle_matrix_Minv(double *out)
{
    memcpy(out, MINV, sizeof MINV);
}

void oracle_matrix_N(double ux, double uy, double *out)
{
    double N[Q][Q];
    shift_matrix(ux, uy, N);
    memcpy(out, N, sizeof N);
}

void oracle_matrix_Ninv(double ux, double uy, double *out)
{
    double NI[Q][Q];
    shift_matrix_inverse(ux, uy, NI);
    memcpy(out, NI, sizeof NI);
}

/* Delta f_i of Sec. III A (Eq. 18) at velocity u. */
void oracle_premnath_delta_f(double Fx, double Fy, double ux, double uy, double *out)
{
    premnath_delta_f(Fx, Fy, ux, uy, out);
}

/* One collision at one node (see collide()). */
void oracle_collide(const double *f, double Fx, double Fy, const double *s6,
                    int scheme, int shift, double *fout)
{
    collide(f, Fx, Fy, s6, scheme, shift, fout);
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * One time step of a whole lattice: collision at every node, then
 * streaming (Eq. 10) in push form.  x is periodic; y is periodic
 * (bc_y = 0) or closed by half-way bounce-back walls half a link below
 * row 0 and above row ny-1 (bc_y = 1).
 *   fin   pre-collision f(x, t)     [9][ny][nx]
 *   fout  pre-collision f(x, t+1)   [9][ny][nx]  (must not alias fin)
 *   fx,fy force density per node    [ny][nx]
 */
int oracle_step(int nx, int ny, int bc_y, const double *s6, int scheme,
                const double *fx, const double *fy, const double *fin,
                double *fout, int nthreads)
{
    if (nx <= 0 || ny <= 0 || !fin || !fout || fin == fout || !fx || !fy) return -1;
    set_threads(nthreads);
    const int64_t plane = (int64_t)nx * ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            const int64_t node = (int64_t)y * nx + x;
            double f[Q], fs[Q];
            for (int i = 0; i < Q; ++i) f[i] = fin[i * plane + node];
            collide(f, fx[node], fy[node], s6, scheme, 1, fs);
            for (int i = 0; i < Q; ++i) {
                const int tx = ((x + EX[i]) % nx + nx) % nx;
                const int ty = y + EY[i];
                if (ty < 0 || ty >= ny) {
                    if (bc_y == 1) {
                        /* Half-way bounce-back: the population returns to
                         * the node it left, reversed. */
                        fout[OPP[i] * plane + node] = fs[i];
                    } else {
                        const int tyw = (ty + ny) % ny;
                        fout[i * plane + (int64_t)tyw * nx + tx] = fs[i];
                    }
                } else {
                    fout[i * plane + (int64_t)ty * nx + tx] = fs[i];
                }
            }
        }
    }
    return 0;
}

/* nsteps steps; f holds f(x,t) on entry and f(x,t+nsteps) on exit; work is
 * a second array of the same size. */
int oracle_run(int nx, int ny, int bc_y, const double *s6, int scheme,
               const double *fx, const double *fy, double *f, double *work,
               int64_t nsteps, int nthreads)
{
    const int64_t n = (int64_t)Q * nx * ny;
    double *a = f, *b = work;
    for (int64_t t = 0; t < nsteps; ++t) {
        int rc = oracle_step(nx, ny, bc_y, s6, scheme, fx, fy, a, b, nthreads);
        if (rc) return rc;
        double *tmp = a;
        a = b;
        b = tmp;
    }
    if (a != f) memcpy(f, a, sizeof(double) * n);
    return 0;
}

/*
 * Initial pre-collision state: f = M^-1 N^-1(u) [rho, -Fx/2, -Fy/2,
 * 2 rho cs^2, 0, 0, 0, 0, rho cs^4] at every node, so that Eq. (15) gives
 * back the requested u.
 */
int oracle_init(int nx, int ny, const double *rho, const double *ux,
                const double *uy, const double *fx, const double *fy, double *f)
{
    if (nx <= 0 || ny <= 0) return -1;
    const int64_t plane = (int64_t)nx * ny;
#pragma omp parallel for schedule(static)
    for (int64_t node = 0; node < plane; ++node) {
        const double r = rho[node];
        const double Tt[Q] = {r, -0.5 * fx[node], -0.5 * fy[node], 2.0 * r * CS2, 0, 0, 0, 0,
                              r * CS2 * CS2};
        double NI[Q][Q], T[Q], fi[Q];
        shift_matrix_inverse(ux[node], uy[node], NI);
        matvec(NI, Tt, T);
        matvec(MINV, T, fi);
        for (int i = 0; i < Q; ++i) f[i * plane + node] = fi[i];
    }
    return 0;
}

/* Density (Eq. 11) and forced velocity (Eq. 15) of a pre-collision state. */
int oracle_moments(int nx, int ny, const double *f, const double *fx,
                   const double *fy, double *rho, double *ux, double *uy)
{
    if (nx <= 0 || ny <= 0) return -1;
    const int64_t plane = (int64_t)nx * ny;
#pragma omp parallel for schedule(static)
    for (int64_t node = 0; node < plane; ++node) {
        double r = 0.0, jx = 0.0, jy = 0.0;
        for (int i = 0; i < Q; ++i) {
            const double v = f[i * plane + node];
            r += v;
            jx += v * EX[i];
            jy += v * EY[i];
        }
        rho[node] = r;
        ux[node] = (jx + 0.5 * fx[node]) / r;
        uy[node] = (jy + 0.5 * fy[node]) / r;
    }
    return 0;
}
