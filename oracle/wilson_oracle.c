/*
 * Plain FP64 CPU oracle of the Wilson hopping term -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * may load this file's library.  The product path (the HIP library) neither
 * links, includes nor calls anything here, and shares no code, header, table
 * or constant with it.
 *
 * What it computes (paper Sec. 2, Eq. (1)):
 *
 *   psi(x) = sum_{mu=0..3} [ U_mu(x) (1 - gamma_mu) phi(x + mu)
 *                          + U_mu(x - mu)^dagger (1 + gamma_mu) phi(x - mu) ]
 *
 * written out literally: for every site and every direction the full 4x4 spin
 * matrix (1 -/+ gamma_mu) is applied to all four spin components of the
 * neighbouring spinor, and then the 3x3 colour matrix U_mu(x) (forward hop) or
 * U_mu(x - mu)^dagger (backward hop) to each of the four resulting colour
 * vectors.  The half-spinor shortcut of Eq. (2) is deliberately not used, so
 * that this route and the GPU route differ algebraically.
 *
 * With dagger != 0 it computes the adjoint operator, i.e. Eq. (1) with the two
 * projectors exchanged: (1 + gamma_mu) on the forward and (1 - gamma_mu) on the
 * backward neighbour.
 *
 * Readings where the paper is silent:
 *  - gamma basis: the chiral basis, gamma_mu block off-diagonal with
 *    upper-right block A_mu = (-i s1, -i s2, -i s3, -1) for mu = x, y, z, t
 *    (s_k the Pauli matrices) and lower-left block A_mu^dagger; it is the basis
 *    in which the statement after Eq. (2), that only two spin components of the
 *    projected spinor are independent, holds for every mu.  The matrices below
 *    are typed in element by element.
 *  - direction mu = 0, 1, 2, 3 is x, y, z, t; site index
 *    lex = x + Lx (y + Ly (z + Lz t)).
 *  - boundary phases: a hop that wraps around the lattice in direction mu picks
 *    up the complex factor z_mu (forward hop from x_mu = L_mu - 1) or conj(z_mu)
 *    (backward hop from x_mu = 0); all other hops carry no phase.
 *
 * Memory layout (canonical, array-of-structures, complex interleaved):
 *   spinor  [lex][spin 4][colour 3]
 *   gauge   [lex][mu 4][row 3][col 3]
 */
#include <complex.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double _Complex cplx;

/* gamma_mu in the chiral basis, rows then columns. */
static const cplx GAMMA[4][4][4] = {
    /* gamma_x */
    {{0, 0, 0, -I}, {0, 0, -I, 0}, {0, I, 0, 0}, {I, 0, 0, 0}},
    /* gamma_y */
    {{0, 0, 0, -1}, {0, 0, 1, 0}, {0, 1, 0, 0}, {-1, 0, 0, 0}},
    /* gamma_z */
    {{0, 0, -I, 0}, {0, 0, 0, I}, {I, 0, 0, 0}, {0, -I, 0, 0}},
    /* gamma_t */
    {{0, 0, -1, 0}, {0, 0, 0, -1}, {-1, 0, 0, 0}, {0, -1, 0, 0}},
};

/* Copy gamma_mu (4x4 complex, row-major, re/im interleaved) to out[32]. */
void orc_gamma(int mu, double *out)
{
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            out[2 * (4 * a + b)] = creal(GAMMA[mu][a][b]);
            out[2 * (4 * a + b) + 1] = cimag(GAMMA[mu][a][b]);
        }
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/*
 * out = H in  (dagger == 0)   or   out = H^dagger in  (dagger != 0)
 * on the full lattice.  in/out: V*12 complex; gauge: V*36 complex;
 * phase: 4 complex (re/im interleaved), phase of a wrapped forward hop.
 */
void orc_hopping(double *out_, const double *in_, const double *gauge_,
                 const int dims[4], const double *phase_, int dagger)
{
    cplx *out = (cplx *)out_;
    const cplx *in = (const cplx *)in_;
    const cplx *gauge = (const cplx *)gauge_;
    const int L[4] = {dims[0], dims[1], dims[2], dims[3]};
    const long vol = (long)L[0] * L[1] * L[2] * L[3];
    cplx z[4];
    for (int mu = 0; mu < 4; ++mu)
        z[mu] = phase_[2 * mu] + I * phase_[2 * mu + 1];
    /* sign of gamma in the forward projector: (1 - s gamma) forward, (1 + s gamma) backward */
    const double s = dagger ? -1.0 : 1.0;

#pragma omp parallel for schedule(static)
    for (long site = 0; site < vol; ++site) {
        int c[4];
        long rem = site;
        for (int mu = 0; mu < 4; ++mu) {
            c[mu] = (int)(rem % L[mu]);
            rem /= L[mu];
        }
        cplx acc[4][3];
        for (int a = 0; a < 4; ++a)
            for (int i = 0; i < 3; ++i)
                acc[a][i] = 0;

        for (int mu = 0; mu < 4; ++mu) {
            /* ---- forward neighbour x + mu ---- */
            int cf[4] = {c[0], c[1], c[2], c[3]};
            cplx ph = 1;
            cf[mu] += 1;
            if (cf[mu] == L[mu]) {
                cf[mu] = 0;
                ph = z[mu];
            }
            long fwd = cf[0] + (long)L[0] * (cf[1] + (long)L[1] * (cf[2] + (long)L[2] * cf[3]));
            /* proj = (1 - s gamma_mu) phi(x + mu), all four spin components */
            cplx proj[4][3];
            for (int a = 0; a < 4; ++a)
                for (int i = 0; i < 3; ++i) {
                    cplx v = in[(fwd * 4 + a) * 3 + i];
                    for (int b = 0; b < 4; ++b)
                        v -= s * GAMMA[mu][a][b] * in[(fwd * 4 + b) * 3 + i];
                    proj[a][i] = v;
                }
            /* acc += phase * U_mu(x) proj, each spin component */
            const cplx *u = gauge + (site * 4 + mu) * 9;
            for (int a = 0; a < 4; ++a)
                for (int i = 0; i < 3; ++i) {
                    cplx v = 0;
                    for (int j = 0; j < 3; ++j)
                        v += u[3 * i + j] * proj[a][j];
                    acc[a][i] += ph * v;
                }

            /* ---- backward neighbour x - mu ---- */
            int cb[4] = {c[0], c[1], c[2], c[3]};
            ph = 1;
            cb[mu] -= 1;
            if (cb[mu] < 0) {
                cb[mu] = L[mu] - 1;
                ph = conj(z[mu]);
            }
            long bwd = cb[0] + (long)L[0] * (cb[1] + (long)L[1] * (cb[2] + (long)L[2] * cb[3]));
            /* proj = (1 + s gamma_mu) phi(x - mu) */
            for (int a = 0; a < 4; ++a)
                for (int i = 0; i < 3; ++i) {
                    cplx v = in[(bwd * 4 + a) * 3 + i];
                    for (int b = 0; b < 4; ++b)
                        v += s * GAMMA[mu][a][b] * in[(bwd * 4 + b) * 3 + i];
                    proj[a][i] = v;
                }
            /* acc += phase * U_mu(x - mu)^dagger proj */
            const cplx *ub = gauge + (bwd * 4 + mu) * 9;
            for (int a = 0; a < 4; ++a)
                for (int i = 0; i < 3; ++i) {
                    cplx v = 0;
                    for (int j = 0; j < 3; ++j)
                        v += conj(ub[3 * j + i]) * proj[a][j];
                    acc[a][i] += ph * v;
                }
        }
        for (int a = 0; a < 4; ++a)
            for (int i = 0; i < 3; ++i)
                out[(site * 4 + a) * 3 + i] = acc[a][i];
    }
}
