/*
 * FP64 reference time stepper for the fictitious-wave-domain Maxwell
 * equations (oracle; TEST INFRASTRUCTURE ONLY, never linked into the
 * product library).
 *
 * Plain loops in the order of the paper's Algorithm 1, one operation per
 * loop nest, no tiling or fusion:
 *   curl H with CPML memory variables (Section 3.4 / 3.1, eqs. HFD2)
 *   inject the electric dipole current J^{n+1/2}
 *   update E:   E^{n+1} = E^n + dt eps^-1 (curl H - J)      (Section 3.1)
 *   record E^{n+1} and H^{n+1/2} at the receivers and add them to the
 *   running DTFT with exp(i omega' t) at each field's own time stamp
 *                                                             (Section 3.5)
 *   curl E with CPML memory variables (eqs. HFD1)
 *   update H:   H^{n+3/2} = H^{n+1/2} - dt mu^-1 curl E       (Section 3.1)
 * OpenMP over the slowest (z) index only.
 *
 * Layout: every 3D array is [n3][n2][n1], x fastest (Section 3.8).
 * Staggering: E1 (i+1/2,j,k), E2 (i,j+1/2,k), E3 (i,j,k+1/2),
 *             H1 (i,j+1/2,k+1/2), H2 (i+1/2,j,k+1/2), H3 (i+1/2,j+1/2,k).
 * D- at integer node i: sum_m cm[i][m] v[i-r+m]      (half nodes i-r..i+r-1)
 * D+ at half node i+1/2: sum_m cp[i][m] u[i-r+1+m]   (nodes i-r+1..i+r)
 * Only cells with every index in [r, n-1-r] are updated; the rest stay 0.
 * CPML memory variables exist where an index is < nb or > n-1-nb on the
 * derivative's own axis (the slab test of Section 3.4); they are stored
 * full-size here for plainness.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int n1, n2, n3;            /* padded sizes */
    int r, nb, nt;
    double ch;                 /* dt / mu0 */
    const double *ce1, *ce2, *ce3;     /* dt / eps at E1/E2/E3 positions */
    const double *cm1, *cm2, *cm3;     /* D- tables [n_d][2r] */
    const double *cp1, *cp2, *cp3;     /* D+ tables [n_d][2r] */
    const double *a1i, *b1i, *a2i, *b2i, *a3i, *b3i;   /* CPML at integer nodes */
    const double *a1h, *b1h, *a2h, *b2h, *a3h, *b3h;   /* CPML at half nodes */
    /* source: component 0..2 (E1..E3 grid), base index, (2r)^3 moment*w/V */
    int src_comp;
    int src_base[3];
    const double *src_q;       /* [2r][2r][2r] (z, y, x) */
    const double *wavelet;     /* s_n, n = 0..nt-1 */
    /* receivers: nrec x nchan stencils */
    int nrec, nchan;
    const int *chan;           /* [nchan] channel ids 0..5 = Ex..Hz */
    const int *rec_base;       /* [nrec][nchan][3] */
    const double *rec_w;       /* [nrec][nchan][2r][2r][2r] (z, y, x) */
    int nfreq;
    const double *phE_re, *phE_im;   /* [nt][nfreq] exp(i w' (n+1) dt) */
    const double *phH_re, *phH_im;   /* [nt][nfreq] exp(i w' (n+1/2) dt) */
    double *acc_re, *acc_im;   /* [nrec][nchan][nfreq] out */
    int nthreads;
    /* first updated z plane: r, or the sea-surface node when the air above
     * it is handled by ghost planes (Section 3.3) */
    int kmin;
    /* called after every E update (which = 0) and H update (which = 1) with
     * the six fields {E1, E2, E3, H1, H2, H3}; fills the ghost planes above
     * kmin (NULL: none) */
    void (*ghost)(int which, double **fields);
    /* lowest-frequency convergence stop (conv_tol > 0; Sections 3.5, 4.1):
     * the DTFT at frequency index conv_f of E1 at 8 corner nodes, compared
     * every conv_every steps with its value at the previous check; the run
     * stops once, for the largest corner change d and magnitude a,
     * 0 < a and d <= conv_tol a */
    double conv_tol;
    int conv_every, conv_f;
    const int *corner;         /* [8][3]: (i, j, k) of E1 */
    int *nt_done;              /* out: steps run (NULL: not reported) */
    double *conv_measure;      /* out: d / a at every check made (NULL: not kept) */
} oracle_params;

#define IDX(k, j, i) (((size_t)(k) * n2 + (size_t)(j)) * n1 + (size_t)(i))

static int in_slab(int i, int n, int nb) { return i < nb || i > n - 1 - nb; }

/* curl H at the E positions, CPML applied (Section 3.4 memory variables) */
static void curl_h(const oracle_params *p, const double *H1, const double *H2,
                   const double *H3, double *c1, double *c2, double *c3,
                   double *mD2H3, double *mD3H2, double *mD3H1,
                   double *mD1H3, double *mD1H2, double *mD2H1)
{
    const int n1 = p->n1, n2 = p->n2, n3 = p->n3, r = p->r, nb = p->nb;
#pragma omp parallel for num_threads(p->nthreads) schedule(static)
    for (int k = p->kmin; k <= n3 - 1 - r; k++) {
        for (int j = r; j <= n2 - 1 - r; j++) {
            for (int i = r; i <= n1 - 1 - r; i++) {
                double D2H3 = 0, D3H2 = 0, D3H1 = 0, D1H3 = 0, D1H2 = 0, D2H1 = 0;
                for (int m = 0; m < 2 * r; m++) {
                    D2H3 += p->cm2[j * 2 * r + m] * H3[IDX(k, j - r + m, i)];
                    D2H1 += p->cm2[j * 2 * r + m] * H1[IDX(k, j - r + m, i)];
                    D3H2 += p->cm3[k * 2 * r + m] * H2[IDX(k - r + m, j, i)];
                    D3H1 += p->cm3[k * 2 * r + m] * H1[IDX(k - r + m, j, i)];
                    D1H3 += p->cm1[i * 2 * r + m] * H3[IDX(k, j, i - r + m)];
                    D1H2 += p->cm1[i * 2 * r + m] * H2[IDX(k, j, i - r + m)];
                }
                size_t id = IDX(k, j, i);
                if (in_slab(i, n1, nb)) {
                    mD1H3[id] = p->b1i[i] * mD1H3[id] + p->a1i[i] * D1H3;
                    mD1H2[id] = p->b1i[i] * mD1H2[id] + p->a1i[i] * D1H2;
                    D1H3 += mD1H3[id];
                    D1H2 += mD1H2[id];
                }
                if (in_slab(j, n2, nb)) {
                    mD2H3[id] = p->b2i[j] * mD2H3[id] + p->a2i[j] * D2H3;
                    mD2H1[id] = p->b2i[j] * mD2H1[id] + p->a2i[j] * D2H1;
                    D2H3 += mD2H3[id];
                    D2H1 += mD2H1[id];
                }
                if (in_slab(k, n3, nb)) {
                    mD3H2[id] = p->b3i[k] * mD3H2[id] + p->a3i[k] * D3H2;
                    mD3H1[id] = p->b3i[k] * mD3H1[id] + p->a3i[k] * D3H1;
                    D3H2 += mD3H2[id];
                    D3H1 += mD3H1[id];
                }
                c1[id] = D2H3 - D3H2;
                c2[id] = D3H1 - D1H3;
                c3[id] = D1H2 - D2H1;
            }
        }
    }
}

/* curl E at the H positions, CPML applied */
static void curl_e(const oracle_params *p, const double *E1, const double *E2,
                   const double *E3, double *c1, double *c2, double *c3,
                   double *mD2E3, double *mD3E2, double *mD3E1,
                   double *mD1E3, double *mD1E2, double *mD2E1)
{
    const int n1 = p->n1, n2 = p->n2, n3 = p->n3, r = p->r, nb = p->nb;
#pragma omp parallel for num_threads(p->nthreads) schedule(static)
    for (int k = p->kmin; k <= n3 - 1 - r; k++) {
        for (int j = r; j <= n2 - 1 - r; j++) {
            for (int i = r; i <= n1 - 1 - r; i++) {
                double D2E3 = 0, D3E2 = 0, D3E1 = 0, D1E3 = 0, D1E2 = 0, D2E1 = 0;
                for (int m = 0; m < 2 * r; m++) {
                    D2E3 += p->cp2[j * 2 * r + m] * E3[IDX(k, j - r + 1 + m, i)];
                    D2E1 += p->cp2[j * 2 * r + m] * E1[IDX(k, j - r + 1 + m, i)];
                    D3E2 += p->cp3[k * 2 * r + m] * E2[IDX(k - r + 1 + m, j, i)];
                    D3E1 += p->cp3[k * 2 * r + m] * E1[IDX(k - r + 1 + m, j, i)];
                    D1E3 += p->cp1[i * 2 * r + m] * E3[IDX(k, j, i - r + 1 + m)];
                    D1E2 += p->cp1[i * 2 * r + m] * E2[IDX(k, j, i - r + 1 + m)];
                }
                size_t id = IDX(k, j, i);
                if (in_slab(i, n1, nb)) {
                    mD1E3[id] = p->b1h[i] * mD1E3[id] + p->a1h[i] * D1E3;
                    mD1E2[id] = p->b1h[i] * mD1E2[id] + p->a1h[i] * D1E2;
                    D1E3 += mD1E3[id];
                    D1E2 += mD1E2[id];
                }
                if (in_slab(j, n2, nb)) {
                    mD2E3[id] = p->b2h[j] * mD2E3[id] + p->a2h[j] * D2E3;
                    mD2E1[id] = p->b2h[j] * mD2E1[id] + p->a2h[j] * D2E1;
                    D2E3 += mD2E3[id];
                    D2E1 += mD2E1[id];
                }
                if (in_slab(k, n3, nb)) {
                    mD3E2[id] = p->b3h[k] * mD3E2[id] + p->a3h[k] * D3E2;
                    mD3E1[id] = p->b3h[k] * mD3E1[id] + p->a3h[k] * D3E1;
                    D3E2 += mD3E2[id];
                    D3E1 += mD3E1[id];
                }
                c1[id] = D2E3 - D3E2;
                c2[id] = D3E1 - D1E3;
                c3[id] = D1E2 - D2E1;
            }
        }
    }
}

static void update(const oracle_params *p, double *F, const double *coef,
                   double scalar, const double *curl, double sign)
{
    const int n1 = p->n1, n2 = p->n2, n3 = p->n3, r = p->r;
#pragma omp parallel for num_threads(p->nthreads) schedule(static)
    for (int k = p->kmin; k <= n3 - 1 - r; k++)
        for (int j = r; j <= n2 - 1 - r; j++)
            for (int i = r; i <= n1 - 1 - r; i++) {
                size_t id = IDX(k, j, i);
                double c = coef ? coef[id] : scalar;
                F[id] += sign * c * curl[id];
            }
}

static double gather(const oracle_params *p, const double *F, const int *base,
                     const double *w)
{
    const int n1 = p->n1, n2 = p->n2, L = 2 * p->r;
    double u = 0.0;
    for (int c = 0; c < L; c++)
        for (int b = 0; b < L; b++)
            for (int a = 0; a < L; a++)
                u += w[(c * L + b) * L + a] *
                     F[IDX(base[2] + c, base[1] + b, base[0] + a)];
    return u;
}

/* Run nt steps from zero fields; accumulate the receiver DTFT. Returns 0, or
 * 1 if any accumulator is non-finite, or -1 on allocation failure. */
int oracle_run(const oracle_params *p)
{
    const int n1 = p->n1, n2 = p->n2, n3 = p->n3, L = 2 * p->r;
    const size_t N = (size_t)n1 * n2 * n3;
    const int nf = p->nfreq;
    /* 6 fields, 6 curls, 12 CPML memory variables */
    double *buf = calloc(24 * N, sizeof(double));
    if (!buf) return -1;
    double *E1 = buf, *E2 = buf + N, *E3 = buf + 2 * N;
    double *H1 = buf + 3 * N, *H2 = buf + 4 * N, *H3 = buf + 5 * N;
    double *c1 = buf + 6 * N, *c2 = buf + 7 * N, *c3 = buf + 8 * N;
    double *m = buf + 9 * N;  /* m[0..5]: curl-H memories, m[6..11]: curl-E */
    double *E[3] = {E1, E2, E3}, *H[3] = {H1, H2, H3}, *cH[3] = {c1, c2, c3};
    double *F6[6] = {E1, E2, E3, H1, H2, H3};
    memset(p->acc_re, 0, sizeof(double) * p->nrec * p->nchan * nf);
    memset(p->acc_im, 0, sizeof(double) * p->nrec * p->nchan * nf);
    double cre[8] = {0}, cim[8] = {0}, pre[8] = {0}, pim[8] = {0};
    int done = p->nt;

    for (int n = 0; n < p->nt; n++) {
        curl_h(p, H1, H2, H3, c1, c2, c3, m, m + N, m + 2 * N, m + 3 * N,
               m + 4 * N, m + 5 * N);
        /* inject: curl H - J at the (2r)^3 support of the source component */
        {
            double *cc = cH[p->src_comp];
            const int *b = p->src_base;
            for (int c = 0; c < L; c++)
                for (int bb = 0; bb < L; bb++)
                    for (int a = 0; a < L; a++)
                        cc[IDX(b[2] + c, b[1] + bb, b[0] + a)] -=
                            p->wavelet[n] * p->src_q[(c * L + bb) * L + a];
        }
        update(p, E1, p->ce1, 0.0, c1, 1.0);
        update(p, E2, p->ce2, 0.0, c2, 1.0);
        update(p, E3, p->ce3, 0.0, c3, 1.0);
        if (p->ghost) p->ghost(0, F6);
        /* record E^{n+1} (stamp (n+1) dt) and H^{n+1/2} (stamp (n+1/2) dt) */
        for (int ir = 0; ir < p->nrec; ir++)
            for (int ic = 0; ic < p->nchan; ic++) {
                int ch = p->chan[ic];
                size_t s = (size_t)ir * p->nchan + ic;
                const double *F = ch < 3 ? E[ch] : H[ch - 3];
                double u = gather(p, F, p->rec_base + 3 * s, p->rec_w + s * L * L * L);
                const double *pr = ch < 3 ? p->phE_re : p->phH_re;
                const double *pi = ch < 3 ? p->phE_im : p->phH_im;
                for (int f = 0; f < nf; f++) {
                    p->acc_re[s * nf + f] += u * pr[(size_t)n * nf + f];
                    p->acc_im[s * nf + f] += u * pi[(size_t)n * nf + f];
                }
            }
        curl_e(p, E1, E2, E3, c1, c2, c3, m + 6 * N, m + 7 * N, m + 8 * N,
               m + 9 * N, m + 10 * N, m + 11 * N);
        update(p, H1, NULL, p->ch, c1, -1.0);
        update(p, H2, NULL, p->ch, c2, -1.0);
        update(p, H3, NULL, p->ch, c3, -1.0);
        if (p->ghost) p->ghost(1, F6);
        if (p->conv_tol > 0.0) {
            const size_t ph = (size_t)n * nf + p->conv_f;
            for (int c = 0; c < 8; c++) {
                const int *q = p->corner + 3 * c;
                const double u = E1[IDX(q[2], q[1], q[0])];
                cre[c] += u * p->phE_re[ph];
                cim[c] += u * p->phE_im[ph];
            }
            if ((n + 1) % p->conv_every == 0) {
                double d = 0.0, a = 0.0;
                for (int c = 0; c < 8; c++) {
                    d = fmax(d, hypot(cre[c] - pre[c], cim[c] - pim[c]));
                    a = fmax(a, hypot(cre[c], cim[c]));
                    pre[c] = cre[c];
                    pim[c] = cim[c];
                }
                if (p->conv_measure) p->conv_measure[(n + 1) / p->conv_every - 1] = a > 0.0 ? d / a : 1.0;
                if (a > 0.0 && d <= p->conv_tol * a) {
                    done = n + 1;
                    break;
                }
            }
        }
    }
    if (p->nt_done) *p->nt_done = done;
    free(buf);
    for (size_t s = 0; s < (size_t)p->nrec * p->nchan * nf; s++)
        if (!isfinite(p->acc_re[s]) || !isfinite(p->acc_im[s])) return 1;
    return 0;
}

/* One curl evaluation on given fields (no CPML state carried): used by the
 * plane-wave symbol tests to pin the stencil offsets of the stepper itself. */
void oracle_curl_h(const oracle_params *p, const double *H1, const double *H2,
                   const double *H3, double *c1, double *c2, double *c3)
{
    size_t N = (size_t)p->n1 * p->n2 * p->n3;
    double *m = calloc(6 * N, sizeof(double));
    curl_h(p, H1, H2, H3, c1, c2, c3, m, m + N, m + 2 * N, m + 3 * N, m + 4 * N, m + 5 * N);
    free(m);
}

void oracle_curl_e(const oracle_params *p, const double *E1, const double *E2,
                   const double *E3, double *c1, double *c2, double *c3)
{
    size_t N = (size_t)p->n1 * p->n2 * p->n3;
    double *m = calloc(6 * N, sizeof(double));
    curl_e(p, E1, E2, E3, c1, c2, c3, m, m + N, m + 2 * N, m + 3 * N, m + 4 * N, m + 5 * N);
    free(m);
}

/* ------------------------------------------------------------------------
 * Discrete adjoint of oracle_run (reverse-mode differentiation written out
 * by hand, FP64).  The misfit chi depends on the receiver DTFT values; its
 * derivative with respect to the real sample u_n of item s is
 *   dchi/du_n = sum_f Re( A[s][f] * exp(i w'_f t_n) ),
 * with A supplied by the caller (for chi = 1/2 sum |log(G/G_obs)|^2 it is
 * conj(r_f)/acc_f).  Output: grad[c][cell] = dchi/d log(dt/eps_c) on the
 * padded grid = sum_n Ebar^{n+1} (E^{n+1} - E^n), because E^{n+1} - E^n is
 * (dt/eps) times the curl term.  Forward states are recomputed per segment
 * of `ckpt` steps from full-state checkpoints.
 *
 * Reverse of one step n (operations of the forward step in reverse order):
 *   H update:  ebar_a = -/+ ch Hbar ;  CPML: psibar = b Q + ebar, ebar += a psibar,
 *              Q = psibar ;  Ebar += (D+)^T ebar
 *   records:   Ebar^{n+1} += w dchi/du (E channels), Hbar^{n+1/2} += w dchi/du (H)
 *   E update:  grad += Ebar (E^{n+1} - E^n) ;  cbar = ce Ebar ; dbar from the
 *              curl signs ; CPML as above ;  Hbar += (D-)^T dbar
 * The transposes are gathers over the per-cell derivative adjoints:
 *   ((D-)^T v)[i'] = sum_m cm[i' + r - 1 - m... ] -- written out below.
 * ------------------------------------------------------------------------ */
static void save_state(const double *buf, double *ck, size_t N) { memcpy(ck, buf, 18 * N * sizeof(double)); }

/* forward step n on state buffer (same order and arithmetic as oracle_run,
 * without the receiver records) */
static void forward_step(const oracle_params *p, double *buf, int n)
{
    const int n1 = p->n1, n2 = p->n2, L = 2 * p->r;
    const size_t N = (size_t)n1 * n2 * p->n3;
    double *E1 = buf, *E2 = buf + N, *E3 = buf + 2 * N;
    double *H1 = buf + 3 * N, *H2 = buf + 4 * N, *H3 = buf + 5 * N;
    double *m = buf + 6 * N;                    /* 12 memory variables */
    double *c1 = buf + 18 * N, *c2 = buf + 19 * N, *c3 = buf + 20 * N;
    double *cH[3] = {c1, c2, c3};
    curl_h(p, H1, H2, H3, c1, c2, c3, m, m + N, m + 2 * N, m + 3 * N, m + 4 * N, m + 5 * N);
    {
        double *cc = cH[p->src_comp];
        const int *b = p->src_base;
        for (int c = 0; c < L; c++)
            for (int bb = 0; bb < L; bb++)
                for (int a = 0; a < L; a++)
                    cc[IDX(b[2] + c, b[1] + bb, b[0] + a)] -=
                        p->wavelet[n] * p->src_q[(c * L + bb) * L + a];
    }
    update(p, E1, p->ce1, 0.0, c1, 1.0);
    update(p, E2, p->ce2, 0.0, c2, 1.0);
    update(p, E3, p->ce3, 0.0, c3, 1.0);
    curl_e(p, E1, E2, E3, c1, c2, c3, m + 6 * N, m + 7 * N, m + 8 * N, m + 9 * N, m + 10 * N, m + 11 * N);
    update(p, H1, NULL, p->ch, c1, -1.0);
    update(p, H2, NULL, p->ch, c2, -1.0);
    update(p, H3, NULL, p->ch, c3, -1.0);
}

/* CPML reverse for one derivative adjoint in place: psibar = b Q + dbar,
 * dbar += a psibar, Q = psibar */
static inline void cpml_rev(double *dbar, double *Q, double a, double b)
{
    double ps = b * (*Q) + *dbar;
    *dbar += a * ps;
    *Q = ps;
}

int oracle_gradient(const oracle_params *p, int ckpt, const double *A_re,
                    const double *A_im, double *grad)
{
    const int n1 = p->n1, n2 = p->n2, n3 = p->n3, r = p->r, L = 2 * r, nb = p->nb;
    const size_t N = (size_t)n1 * n2 * n3;
    const int nt = p->nt, nf = p->nfreq;
    const int nseg = (nt + ckpt - 1) / ckpt;
    if (p->kmin != r || p->ghost) return -2;      /* the adjoint of the air boundary is not built */
    /* working state: 18 N (fields + memories) + 3 N curl scratch */
    double *buf = calloc(21 * N, sizeof(double));
    double *cks = calloc((size_t)nseg * 18 * N, sizeof(double));
    double *seg = calloc((size_t)(ckpt + 1) * 3 * N, sizeof(double));   /* E^n of the segment */
    /* adjoint: Eb[3], Hb[3], Q for the 6 E-step and 6 H-step memories, 6 derivative adjoints */
    double *adj = calloc(24 * N, sizeof(double));
    if (!buf || !cks || !seg || !adj) { free(buf); free(cks); free(seg); free(adj); return -1; }
    double *Eb[3] = {adj, adj + N, adj + 2 * N}, *Hb[3] = {adj + 3 * N, adj + 4 * N, adj + 5 * N};
    double *Qh = adj + 6 * N;     /* 6 arrays: adjoints of the curl-H memories */
    double *Qe = adj + 12 * N;    /* 6 arrays: adjoints of the curl-E memories */
    double *db = adj + 18 * N;    /* 6 arrays: derivative adjoints of the current half step */
    memset(grad, 0, 3 * N * sizeof(double));

    /* forward with checkpoints */
    for (int n = 0; n < nt; n++) {
        if (n % ckpt == 0) save_state(buf, cks + (size_t)(n / ckpt) * 18 * N, N);
        forward_step(p, buf, n);
    }
    for (int sgi = nseg - 1; sgi >= 0; sgi--) {
        const int n0 = sgi * ckpt, nend = (n0 + ckpt < nt) ? n0 + ckpt : nt;
        memcpy(buf, cks + (size_t)sgi * 18 * N, 18 * N * sizeof(double));
        memcpy(seg, buf, 3 * N * sizeof(double));
        for (int n = n0; n < nend; n++) {
            forward_step(p, buf, n);
            memcpy(seg + (size_t)(n - n0 + 1) * 3 * N, buf, 3 * N * sizeof(double));
        }
        for (int n = nend - 1; n >= n0; n--) {
            const double *En = seg + (size_t)(n - n0) * 3 * N;        /* E^n */
            const double *En1 = seg + (size_t)(n - n0 + 1) * 3 * N;   /* E^{n+1} */
            /* --- reverse of the H update: derivative adjoints of curl E --- */
            memset(db, 0, 6 * N * sizeof(double));
#pragma omp parallel for num_threads(p->nthreads) schedule(static)
            for (int k = r; k <= n3 - 1 - r; k++)
                for (int j = r; j <= n2 - 1 - r; j++)
                    for (int i = r; i <= n1 - 1 - r; i++) {
                        size_t id = IDX(k, j, i);
                        /* order: D2E3, D3E2, D3E1, D1E3, D1E2, D2E1 */
                        double d[6] = {-p->ch * Hb[0][id], p->ch * Hb[0][id],
                                       -p->ch * Hb[1][id], p->ch * Hb[1][id],
                                       -p->ch * Hb[2][id], p->ch * Hb[2][id]};
                        if (in_slab(j, n2, nb)) {
                            cpml_rev(&d[0], &Qe[0 * N + id], p->a2h[j], p->b2h[j]);
                            cpml_rev(&d[5], &Qe[5 * N + id], p->a2h[j], p->b2h[j]);
                        }
                        if (in_slab(k, n3, nb)) {
                            cpml_rev(&d[1], &Qe[1 * N + id], p->a3h[k], p->b3h[k]);
                            cpml_rev(&d[2], &Qe[2 * N + id], p->a3h[k], p->b3h[k]);
                        }
                        if (in_slab(i, n1, nb)) {
                            cpml_rev(&d[3], &Qe[3 * N + id], p->a1h[i], p->b1h[i]);
                            cpml_rev(&d[4], &Qe[4 * N + id], p->a1h[i], p->b1h[i]);
                        }
                        for (int q = 0; q < 6; q++) db[q * N + id] = d[q];
                    }
            /* Ebar += (D+)^T dbar: e_{D2E3}[j] = sum_m cp2[j][m] E3[j-r+1+m], so
             * E3[j'] receives cp2[j][m] dbar[j] for every (j, m) with
             * j - r + 1 + m = j', i.e. j = j' + r - 1 - m. */
#pragma omp parallel for num_threads(p->nthreads) schedule(static)
            for (int k = 0; k < n3; k++)
                for (int j = 0; j < n2; j++)
                    for (int i = 0; i < n1; i++) {
                        size_t id = IDX(k, j, i);
                        double e1 = 0, e2 = 0, e3 = 0;
                        for (int m2 = 0; m2 < L; m2++) {
                            int jj = j + r - 1 - m2, kk = k + r - 1 - m2, ii = i + r - 1 - m2;
                            if (jj >= r && jj <= n2 - 1 - r) {
                                double c = p->cp2[jj * L + m2];
                                e3 += c * db[0 * N + IDX(k, jj, i)];     /* D2E3 */
                                e1 += c * db[5 * N + IDX(k, jj, i)];     /* D2E1 */
                            }
                            if (kk >= r && kk <= n3 - 1 - r) {
                                double c = p->cp3[kk * L + m2];
                                e2 += c * db[1 * N + IDX(kk, j, i)];     /* D3E2 */
                                e1 += c * db[2 * N + IDX(kk, j, i)];     /* D3E1 */
                            }
                            if (ii >= r && ii <= n1 - 1 - r) {
                                double c = p->cp1[ii * L + m2];
                                e3 += c * db[3 * N + IDX(k, j, ii)];     /* D1E3 */
                                e2 += c * db[4 * N + IDX(k, j, ii)];     /* D1E2 */
                            }
                        }
                        Eb[0][id] += e1;
                        Eb[1][id] += e2;
                        Eb[2][id] += e3;
                    }
            /* --- records: E^{n+1} at stamp (n+1) dt, H^{n+1/2} at (n+1/2) dt --- */
            for (int ir = 0; ir < p->nrec; ir++)
                for (int ic = 0; ic < p->nchan; ic++) {
                    int ch = p->chan[ic];
                    size_t s = (size_t)ir * p->nchan + ic;
                    const double *pr = ch < 3 ? p->phE_re : p->phH_re;
                    const double *pi = ch < 3 ? p->phE_im : p->phH_im;
                    double g = 0.0;
                    for (int f = 0; f < nf; f++)
                        g += A_re[s * nf + f] * pr[(size_t)n * nf + f] - A_im[s * nf + f] * pi[(size_t)n * nf + f];
                    double *F = ch < 3 ? Eb[ch] : Hb[ch - 3];
                    const int *b = p->rec_base + 3 * s;
                    const double *w = p->rec_w + s * L * L * L;
                    for (int c = 0; c < L; c++)
                        for (int bb = 0; bb < L; bb++)
                            for (int a = 0; a < L; a++)
                                F[IDX(b[2] + c, b[1] + bb, b[0] + a)] += w[(c * L + bb) * L + a] * g;
                }
            /* --- reverse of the E update --- */
            memset(db, 0, 6 * N * sizeof(double));
#pragma omp parallel for num_threads(p->nthreads) schedule(static)
            for (int k = r; k <= n3 - 1 - r; k++)
                for (int j = r; j <= n2 - 1 - r; j++)
                    for (int i = r; i <= n1 - 1 - r; i++) {
                        size_t id = IDX(k, j, i);
                        for (int c = 0; c < 3; c++)
                            grad[c * N + id] += Eb[c][id] * (En1[c * N + id] - En[c * N + id]);
                        double cb1 = p->ce1[id] * Eb[0][id], cb2 = p->ce2[id] * Eb[1][id],
                               cb3 = p->ce3[id] * Eb[2][id];
                        /* order: D2H3, D3H2, D3H1, D1H3, D1H2, D2H1 */
                        double d[6] = {cb1, -cb1, cb2, -cb2, cb3, -cb3};
                        if (in_slab(j, n2, nb)) {
                            cpml_rev(&d[0], &Qh[0 * N + id], p->a2i[j], p->b2i[j]);
                            cpml_rev(&d[5], &Qh[5 * N + id], p->a2i[j], p->b2i[j]);
                        }
                        if (in_slab(k, n3, nb)) {
                            cpml_rev(&d[1], &Qh[1 * N + id], p->a3i[k], p->b3i[k]);
                            cpml_rev(&d[2], &Qh[2 * N + id], p->a3i[k], p->b3i[k]);
                        }
                        if (in_slab(i, n1, nb)) {
                            cpml_rev(&d[3], &Qh[3 * N + id], p->a1i[i], p->b1i[i]);
                            cpml_rev(&d[4], &Qh[4 * N + id], p->a1i[i], p->b1i[i]);
                        }
                        for (int q = 0; q < 6; q++) db[q * N + id] = d[q];
                    }
            /* Hbar += (D-)^T dbar: d_{D2H3}[j] = sum_m cm2[j][m] H3[j-r+m], so
             * H3[j'] receives cm2[j][m] dbar[j] for j = j' + r - m. */
#pragma omp parallel for num_threads(p->nthreads) schedule(static)
            for (int k = 0; k < n3; k++)
                for (int j = 0; j < n2; j++)
                    for (int i = 0; i < n1; i++) {
                        size_t id = IDX(k, j, i);
                        double h1 = 0, h2 = 0, h3 = 0;
                        for (int m2 = 0; m2 < L; m2++) {
                            int jj = j + r - m2, kk = k + r - m2, ii = i + r - m2;
                            if (jj >= r && jj <= n2 - 1 - r) {
                                double c = p->cm2[jj * L + m2];
                                h3 += c * db[0 * N + IDX(k, jj, i)];     /* D2H3 */
                                h1 += c * db[5 * N + IDX(k, jj, i)];     /* D2H1 */
                            }
                            if (kk >= r && kk <= n3 - 1 - r) {
                                double c = p->cm3[kk * L + m2];
                                h2 += c * db[1 * N + IDX(kk, j, i)];     /* D3H2 */
                                h1 += c * db[2 * N + IDX(kk, j, i)];     /* D3H1 */
                            }
                            if (ii >= r && ii <= n1 - 1 - r) {
                                double c = p->cm1[ii * L + m2];
                                h3 += c * db[3 * N + IDX(k, j, ii)];     /* D1H3 */
                                h2 += c * db[4 * N + IDX(k, j, ii)];     /* D1H2 */
                            }
                        }
                        Hb[0][id] += h1;
                        Hb[1][id] += h2;
                        Hb[2][id] += h3;
                    }
        }
    }
    free(buf);
    free(cks);
    free(seg);
    free(adj);
    return 0;
}
