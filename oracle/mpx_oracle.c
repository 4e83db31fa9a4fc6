/*
 * mpx_oracle.c -- plain FP64 CPU oracle for the coupled Yee + LLG time step.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference that the GPU path is
 * checked against; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code, header, table or helper
 * with the HIP library, and it must never be used as a fallback for it.
 *
 * What it computes (arXiv:2510.22221, Methods, "Numerical Model"):
 *   - Ampere's law with conduction, eq. (Ampere), discretised semi-implicitly
 *     in sigma as in the unlabelled E update that closes that subsection;
 *   - Faraday's law with B = mu0 (H + M), eq. (Faraday) and the constitutive
 *     law stated next to it, integrated as eq. (iterate_H);
 *   - the Gilbert-form LLG, eq. (LLG), discretised with the trapezoidal rule
 *     whose closed form is eqs. (llg_tra4)-(llg_tra6), then normalised to Ms;
 *   - M = 0 and a plain Faraday update where Ms = 0 (same subsection, last
 *     sentence).
 * The readings taken where the paper is silent (half-step H/M schedule,
 * where M lives, transverse field at a face, material averaging, CPML,
 * source timing, initial state) are listed in the design notes; each is
 * marked "reading" below.
 *
 * Everything is written as the plain definition: natural Yee index ranges,
 * one loop per update, no blocking, no fusion.  Floating point is double
 * throughout; build with -O2 -ffp-contract=off.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PEC 0
#define ORC_PML 1
#define ORC_PERIODIC 2

#define ORC_PROBE_FIELD 0   /* one field component at one site           */
#define ORC_PROBE_MEAN_M 1  /* film-averaged M, 3 values per sample       */
#define ORC_PROBE_FILM_ENERGY 2

static const double ORC_PI = 3.14159265358979323846;
static const double ORC_C0 = 299792458.0;
/* mu0 = 4 pi 1e-7 H/m, eps0 = 1/(mu0 c^2) */
#define ORC_MU0 (4.0e-7 * ORC_PI)
#define ORC_EPS0 (1.0 / (ORC_MU0 * ORC_C0 * ORC_C0))

typedef struct {
    int32_t nx, ny, nz;
    double dx, dy, dz, dt;
    int32_t bc[6];   /* -x,+x,-y,+y,-z,+z */
    int32_t npml[6];
    double pml_order, pml_sigma_factor;
} orc_grid;

typedef struct {
    double eps_r, sigma;
    int32_t is_pec;
    double Ms, alpha, gamma_abs;
} orc_material;

typedef struct {
    int comp;
    int box[6]; /* i0,j0,k0,ni,nj,nk in E_comp index space */
    double *table;
    int64_t n;
} orc_source;

typedef struct {
    int kind, field, i, j, k, film;
    int nval;
    double *data;
    int64_t n, cap;
} orc_probe;

typedef struct {
    int box[6]; /* cell box: i0,j0,k0,ni,nj,nk */
    int64_t ncells;
    int64_t lowest;
} orc_film;

typedef struct orc_sim {
    orc_grid g;
    int N[3];
    int per[3];
    double d[3];
    int dimE[3][3], dimH[3][3];
    int64_t nE[3], nH[3];
    double *E[3], *H[3];
    /* materials */
    int nmat;
    orc_material mat[256];
    uint8_t *id;
    int have_mat;
    double *ca[3], *cb[3];
    uint8_t *epec[3];
    double *Ms_s[3], *al_s[3], *ga_s[3];
    /* magnetisation: full family arrays, only within k in [mk0[c], mk1[c]) */
    int has_mag;
    int mk0[3], mk1[3]; /* per family */
    double *M[3][3], *M0[3][3];
    double *Mn_tmp[3][3], *Hn_tmp[3];
    double H0[3];
    /* CPML: psiE[c][w], psiH[c][w] over the component's natural dims */
    double *psiE[3][3], *psiH[3][3];
    double *bE[3], *cE[3], *bH[3], *cH[3]; /* per axis: index = integer pos (E) / half pos (H) */
    /* films */
    int nfilm;
    orc_film film[64];
    /* sources / probes */
    int nsrc;
    orc_source src[16];
    int nprobe;
    orc_probe probe[64];
    int64_t step;
    int last_r;
} orc_sim;

/* ------------------------------------------------------------------ */
/* index helpers                                                       */
/* ------------------------------------------------------------------ */

static int64_t lin(const int *dim, int i, int j, int k) {
    return (int64_t)i + (int64_t)dim[0] * ((int64_t)j + (int64_t)dim[1] * k);
}

/* Map an index along axis a of an array with extent n to the stored index:
 * wraps on a periodic axis, returns -1 when outside the domain. */
static int fold(const orc_sim *s, int a, int i, int n) {
    if (s->per[a]) {
        if (i < 0) i += n;
        if (i >= n) i -= n;
        return i;
    }
    if (i < 0 || i >= n) return -1;
    return i;
}

/* value of an array at (i,j,k) with wrap, or 0 (and *ok = 0) outside */
static double at(const orc_sim *s, const double *a, const int *dim, int i, int j, int k, int *ok) {
    int ii = fold(s, 0, i, dim[0]), jj = fold(s, 1, j, dim[1]), kk = fold(s, 2, k, dim[2]);
    if (ii < 0 || jj < 0 || kk < 0) {
        if (ok) *ok = 0;
        return 0.0;
    }
    if (ok) *ok = 1;
    return a[lin(dim, ii, jj, kk)];
}

static int cell_id(const orc_sim *s, int i, int j, int k) {
    int ii = fold(s, 0, i, s->N[0]), jj = fold(s, 1, j, s->N[1]), kk = fold(s, 2, k, s->N[2]);
    if (ii < 0 || jj < 0 || kk < 0) return -1;
    return s->id[lin(s->N, ii, jj, kk)];
}

/* ------------------------------------------------------------------ */
/* creation                                                            */
/* ------------------------------------------------------------------ */

orc_sim *orc_create(const orc_grid *g) {
    if (!g || g->nx < 1 || g->ny < 1 || g->nz < 1 || !(g->dt > 0)) return NULL;
    for (int a = 0; a < 3; a++) {
        int lo = g->bc[2 * a], hi = g->bc[2 * a + 1];
        if ((lo == ORC_PERIODIC) != (hi == ORC_PERIODIC)) return NULL;
    }
    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    s->g = *g;
    s->N[0] = g->nx; s->N[1] = g->ny; s->N[2] = g->nz;
    s->d[0] = g->dx; s->d[1] = g->dy; s->d[2] = g->dz;
    for (int a = 0; a < 3; a++) s->per[a] = (g->bc[2 * a] == ORC_PERIODIC);
    /* Yee index ranges: E_c is half-integer along c, integer along the others;
     * H_c is integer along c, half-integer along the others.  A periodic axis
     * has N integer positions, otherwise N+1. */
    for (int c = 0; c < 3; c++) {
        for (int a = 0; a < 3; a++) {
            int nint = s->N[a] + (s->per[a] ? 0 : 1);
            s->dimE[c][a] = (a == c) ? s->N[a] : nint;
            s->dimH[c][a] = (a == c) ? nint : s->N[a];
        }
        s->nE[c] = (int64_t)s->dimE[c][0] * s->dimE[c][1] * s->dimE[c][2];
        s->nH[c] = (int64_t)s->dimH[c][0] * s->dimH[c][1] * s->dimH[c][2];
        s->E[c] = (double *)calloc(s->nE[c], sizeof(double));
        s->H[c] = (double *)calloc(s->nH[c], sizeof(double));
        s->ca[c] = (double *)calloc(s->nE[c], sizeof(double));
        s->cb[c] = (double *)calloc(s->nE[c], sizeof(double));
        s->epec[c] = (uint8_t *)calloc(s->nE[c], 1);
        s->Ms_s[c] = (double *)calloc(s->nH[c], sizeof(double));
        s->al_s[c] = (double *)calloc(s->nH[c], sizeof(double));
        s->ga_s[c] = (double *)calloc(s->nH[c], sizeof(double));
    }
    int64_t ncell = (int64_t)s->N[0] * s->N[1] * s->N[2];
    s->id = (uint8_t *)calloc(ncell, 1);

    /* CPML grading (reading: convolutional PML, kappa = 1, a = 0,
     * sigma(rho) = sigma_max rho^m, sigma_max = f (m+1)/(eta0 d)).
     * Per axis: arrays indexed by integer position p (E-type derivative)
     * and by half position p+1/2 (H-type derivative). */
    double m = g->pml_order > 0 ? g->pml_order : 3.0;
    double f = g->pml_sigma_factor > 0 ? g->pml_sigma_factor : 0.8;
    double eta0 = sqrt(ORC_MU0 / ORC_EPS0);
    for (int a = 0; a < 3; a++) {
        int n = s->N[a];
        s->bE[a] = (double *)malloc((n + 1) * sizeof(double));
        s->cE[a] = (double *)malloc((n + 1) * sizeof(double));
        s->bH[a] = (double *)malloc((n + 1) * sizeof(double));
        s->cH[a] = (double *)malloc((n + 1) * sizeof(double));
        int nlo = (g->bc[2 * a] == ORC_PML) ? g->npml[2 * a] : 0;
        int nhi = (g->bc[2 * a + 1] == ORC_PML) ? g->npml[2 * a + 1] : 0;
        double smax = f * (m + 1.0) / (eta0 * s->d[a]);
        for (int p = 0; p <= n; p++) {
            for (int half = 0; half < 2; half++) {
                double x = p + 0.5 * half;
                double rho = 0.0;
                if (nlo > 0 && x < nlo) rho = (nlo - x) / nlo;
                if (nhi > 0 && x > n - nhi) rho = (x - (n - nhi)) / nhi;
                double sig = smax * pow(rho, m);
                if (half == 0) {
                    double b = exp(-sig * g->dt / ORC_EPS0);
                    s->bE[a][p] = b;
                    s->cE[a][p] = b - 1.0;
                } else {
                    double b = exp(-sig * (0.5 * g->dt) / ORC_EPS0);
                    s->bH[a][p] = b;
                    s->cH[a][p] = b - 1.0;
                }
            }
        }
        if (nlo > 0 || nhi > 0) {
            for (int c = 0; c < 3; c++) {
                if (c == a) continue;
                s->psiE[c][a] = (double *)calloc(s->nE[c], sizeof(double));
                s->psiH[c][a] = (double *)calloc(s->nH[c], sizeof(double));
            }
        }
    }
    return s;
}

void orc_destroy(orc_sim *s) {
    if (!s) return;
    for (int c = 0; c < 3; c++) {
        free(s->E[c]); free(s->H[c]); free(s->ca[c]); free(s->cb[c]); free(s->epec[c]);
        free(s->Ms_s[c]); free(s->al_s[c]); free(s->ga_s[c]);
        free(s->bE[c]); free(s->cE[c]); free(s->bH[c]); free(s->cH[c]);
        free(s->Hn_tmp[c]);
        for (int w = 0; w < 3; w++) {
            free(s->psiE[c][w]); free(s->psiH[c][w]);
            free(s->M[c][w]); free(s->M0[c][w]); free(s->Mn_tmp[c][w]);
        }
    }
    for (int i = 0; i < s->nsrc; i++) free(s->src[i].table);
    for (int i = 0; i < s->nprobe; i++) free(s->probe[i].data);
    free(s->id);
    free(s);
}

/* ------------------------------------------------------------------ */
/* materials -> coefficients (reading: edges average the <=4 cells     */
/* that share them, faces average the <=2 cells that share them)       */
/* ------------------------------------------------------------------ */

static int in_pml_cell(const orc_sim *s, int a, int i) {
    int nlo = (s->g.bc[2 * a] == ORC_PML) ? s->g.npml[2 * a] : 0;
    int nhi = (s->g.bc[2 * a + 1] == ORC_PML) ? s->g.npml[2 * a + 1] : 0;
    return i < nlo || i >= s->N[a] - nhi;
}

/* connected components of magnetic cells -> bounding boxes; boxes closer
 * than two cells are merged; films are numbered by lowest cell index */
static void find_films(orc_sim *s) {
    int64_t ncell = (int64_t)s->N[0] * s->N[1] * s->N[2];
    int32_t *lab = (int32_t *)malloc(ncell * sizeof(int32_t));
    int64_t *stack = (int64_t *)malloc(ncell * sizeof(int64_t));
    for (int64_t q = 0; q < ncell; q++) lab[q] = -1;
    int nb = 0;
    static int boxes[4096][6];
    static int64_t low[4096];
    for (int64_t q = 0; q < ncell; q++) {
        if (lab[q] >= 0 || !(s->mat[s->id[q]].Ms > 0)) continue;
        if (nb >= 4096) break;
        int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-1, -1, -1};
        int64_t sp = 0;
        stack[sp++] = q;
        lab[q] = nb;
        while (sp) {
            int64_t p = stack[--sp];
            int c[3] = {(int)(p % s->N[0]), (int)((p / s->N[0]) % s->N[1]), (int)(p / ((int64_t)s->N[0] * s->N[1]))};
            for (int a = 0; a < 3; a++) {
                if (c[a] < lo[a]) lo[a] = c[a];
                if (c[a] > hi[a]) hi[a] = c[a];
            }
            for (int a = 0; a < 3; a++)
                for (int sg = -1; sg <= 1; sg += 2) {
                    int nc[3] = {c[0], c[1], c[2]};
                    nc[a] += sg;
                    if (nc[a] < 0 || nc[a] >= s->N[a]) continue; /* no wrap: boxes are plain */
                    int64_t pn = lin(s->N, nc[0], nc[1], nc[2]);
                    if (lab[pn] < 0 && s->mat[s->id[pn]].Ms > 0) {
                        lab[pn] = nb;
                        stack[sp++] = pn;
                    }
                }
        }
        for (int a = 0; a < 3; a++) {
            boxes[nb][a] = lo[a];
            boxes[nb][3 + a] = hi[a] + 1;
        }
        low[nb] = q;
        nb++;
    }
    /* merge boxes whose gap is below two cells on every axis */
    int merged = 1;
    while (merged) {
        merged = 0;
        for (int x = 0; x < nb && !merged; x++)
            for (int y = x + 1; y < nb && !merged; y++) {
                int close = 1;
                for (int a = 0; a < 3; a++) {
                    int gap = boxes[y][a] >= boxes[x][3 + a] ? boxes[y][a] - boxes[x][3 + a]
                              : boxes[x][a] >= boxes[y][3 + a] ? boxes[x][a] - boxes[y][3 + a]
                                                              : 0;
                    if (gap >= 2) close = 0;
                }
                if (close) {
                    for (int a = 0; a < 3; a++) {
                        if (boxes[y][a] < boxes[x][a]) boxes[x][a] = boxes[y][a];
                        if (boxes[y][3 + a] > boxes[x][3 + a]) boxes[x][3 + a] = boxes[y][3 + a];
                    }
                    if (low[y] < low[x]) low[x] = low[y];
                    for (int z = y; z < nb - 1; z++) {
                        memcpy(boxes[z], boxes[z + 1], sizeof(boxes[z]));
                        low[z] = low[z + 1];
                    }
                    nb--;
                    merged = 1;
                }
            }
    }
    /* order by lowest linear cell index */
    for (int x = 0; x < nb; x++)
        for (int y = x + 1; y < nb; y++)
            if (low[y] < low[x]) {
                int tb[6];
                memcpy(tb, boxes[x], sizeof(tb));
                memcpy(boxes[x], boxes[y], sizeof(tb));
                memcpy(boxes[y], tb, sizeof(tb));
                int64_t tl = low[x]; low[x] = low[y]; low[y] = tl;
            }
    s->nfilm = nb < 64 ? nb : 64;
    for (int f = 0; f < s->nfilm; f++) {
        orc_film *F = &s->film[f];
        for (int a = 0; a < 3; a++) {
            F->box[a] = boxes[f][a];
            F->box[3 + a] = boxes[f][3 + a] - boxes[f][a];
        }
        F->lowest = low[f];
        F->ncells = 0;
        for (int k = F->box[2]; k < F->box[2] + F->box[5]; k++)
            for (int j = F->box[1]; j < F->box[1] + F->box[4]; j++)
                for (int i = F->box[0]; i < F->box[0] + F->box[3]; i++)
                    if (s->mat[s->id[lin(s->N, i, j, k)]].Ms > 0) F->ncells++;
    }
    free(lab);
    free(stack);
}

int orc_set_materials(orc_sim *s, const orc_material *tab, int n, const uint8_t *ids) {
    if (!s || !tab || !ids || n < 1 || n > 256) return 1;
    int64_t ncell = (int64_t)s->N[0] * s->N[1] * s->N[2];
    for (int64_t q = 0; q < ncell; q++)
        if (ids[q] >= n) return 1;
    s->nmat = n;
    memcpy(s->mat, tab, n * sizeof(orc_material));
    memcpy(s->id, ids, ncell);

    /* a magnetic cell may not sit in, or next to, a PML slab */
    for (int k = 0; k < s->N[2]; k++)
        for (int j = 0; j < s->N[1]; j++)
            for (int i = 0; i < s->N[0]; i++) {
                if (!(s->mat[s->id[lin(s->N, i, j, k)]].Ms > 0)) continue;
                int c3[3] = {i, j, k};
                for (int a = 0; a < 3; a++)
                    for (int dd = -1; dd <= 1; dd++) {
                        int x = c3[a] + dd;
                        if (x < 0 || x >= s->N[a]) continue;
                        if (in_pml_cell(s, a, x)) return 2;
                    }
            }

    /* E edges: cells sharing E_c(idx) are idx along c and {idx-1, idx}
     * along the two other axes; keep those inside the domain. */
    for (int c = 0; c < 3; c++) {
        int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        const int *dim = s->dimE[c];
        for (int k = 0; k < dim[2]; k++)
            for (int j = 0; j < dim[1]; j++)
                for (int i = 0; i < dim[0]; i++) {
                    int idx[3] = {i, j, k};
                    int64_t q = lin(dim, i, j, k);
                    /* tangential to a non-periodic domain face: held at zero */
                    int wall = 0;
                    for (int a = 0; a < 3; a++)
                        if (a != c && !s->per[a] && (idx[a] == 0 || idx[a] == s->N[a])) wall = 1;
                    double se = 0.0, ss = 0.0;
                    int cnt = 0, pec = wall;
                    for (int u = -1; u <= 0; u++)
                        for (int v = -1; v <= 0; v++) {
                            int cc[3];
                            cc[c] = idx[c];
                            cc[c1] = idx[c1] + u;
                            cc[c2] = idx[c2] + v;
                            int m = cell_id(s, cc[0], cc[1], cc[2]);
                            if (m < 0) continue;
                            se += s->mat[m].eps_r;
                            ss += s->mat[m].sigma;
                            if (s->mat[m].is_pec) pec = 1;
                            cnt++;
                        }
                    s->epec[c][q] = (uint8_t)pec;
                    if (pec || cnt == 0) {
                        s->ca[c][q] = 0.0;
                        s->cb[c][q] = 0.0;
                        continue;
                    }
                    double eps = ORC_EPS0 * (se / cnt);
                    double sig = ss / cnt;
                    /* E^{n+1} = (sigma/2 + eps/dt)^{-1} [curl H - (sigma/2 - eps/dt) E^n - J] */
                    double den = sig / 2.0 + eps / s->g.dt;
                    s->ca[c][q] = -(sig / 2.0 - eps / s->g.dt) / den;
                    s->cb[c][q] = 1.0 / den;
                }
    }
    /* H faces: cells sharing H_c(idx) are {idx-1, idx} along c, idx along
     * the others.  Ms_s is the mean over those inside the domain; alpha and
     * |gamma| are the mean over the magnetic ones among them. */
    int mk0[3], mk1[3];
    for (int c = 0; c < 3; c++) {
        mk0[c] = 1 << 30;
        mk1[c] = -1;
        const int *dim = s->dimH[c];
        for (int k = 0; k < dim[2]; k++)
            for (int j = 0; j < dim[1]; j++)
                for (int i = 0; i < dim[0]; i++) {
                    int idx[3] = {i, j, k};
                    double sm = 0.0, sa = 0.0, sgm = 0.0;
                    int cnt = 0, nm = 0;
                    for (int u = -1; u <= 0; u++) {
                        int cc[3] = {idx[0], idx[1], idx[2]};
                        cc[c] += u;
                        int m = cell_id(s, cc[0], cc[1], cc[2]);
                        if (m < 0) continue;
                        cnt++;
                        sm += s->mat[m].Ms;
                        if (s->mat[m].Ms > 0) {
                            nm++;
                            sa += s->mat[m].alpha;
                            sgm += s->mat[m].gamma_abs;
                        }
                    }
                    int64_t q = lin(dim, i, j, k);
                    s->Ms_s[c][q] = cnt ? sm / cnt : 0.0;
                    s->al_s[c][q] = nm ? sa / nm : 0.0;
                    s->ga_s[c][q] = nm ? sgm / nm : 0.0;
                    if (s->Ms_s[c][q] > 0) {
                        if (k < mk0[c]) mk0[c] = k;
                        if (k + 1 > mk1[c]) mk1[c] = k + 1;
                    }
                }
    }
    for (int c = 0; c < 3; c++) {
        free(s->Hn_tmp[c]);
        s->Hn_tmp[c] = NULL;
        for (int w = 0; w < 3; w++) {
            free(s->M[c][w]); free(s->M0[c][w]); free(s->Mn_tmp[c][w]);
            s->M[c][w] = s->M0[c][w] = s->Mn_tmp[c][w] = NULL;
        }
    }
    s->has_mag = 0;
    for (int c = 0; c < 3; c++) {
        if (mk1[c] <= mk0[c]) mk0[c] = mk1[c] = 0; /* empty range */
        s->mk0[c] = mk0[c];
        s->mk1[c] = mk1[c];
        if (mk1[c] > mk0[c]) s->has_mag = 1;
    }
    if (s->has_mag) {
        for (int c = 0; c < 3; c++) {
            int64_t nplane = (int64_t)s->dimH[c][0] * s->dimH[c][1] * (s->mk1[c] - s->mk0[c]);
            if (nplane < 1) nplane = 1;
            s->Hn_tmp[c] = (double *)calloc(nplane, sizeof(double));
            for (int w = 0; w < 3; w++) {
                s->M[c][w] = (double *)calloc(nplane, sizeof(double));
                s->M0[c][w] = (double *)calloc(nplane, sizeof(double));
                s->Mn_tmp[c][w] = (double *)calloc(nplane, sizeof(double));
            }
        }
    }
    find_films(s);
    s->have_mat = 1;
    return 0;
}

/* index into the magnetisation arrays of family c (restricted k range) */
static int64_t mlin(const orc_sim *s, int c, int i, int j, int k) {
    return (int64_t)i + (int64_t)s->dimH[c][0] * ((int64_t)j + (int64_t)s->dimH[c][1] * (k - s->mk0[c]));
}

void orc_set_bias(orc_sim *s, double hx, double hy, double hz) {
    s->H0[0] = hx; s->H0[1] = hy; s->H0[2] = hz;
}

/* M = Ms_s u at every magnetic site of each family (reading: the paper
 * saturates the film along the bias; the direction is a parameter here). */
int orc_init_magnetization(orc_sim *s, double ux, double uy, double uz) {
    if (!s->have_mat) return 2;
    double nrm = sqrt(ux * ux + uy * uy + uz * uz);
    if (!(nrm > 0)) return 1;
    double u[3] = {ux / nrm, uy / nrm, uz / nrm};
    if (!s->has_mag) return 0;
    for (int c = 0; c < 3; c++) {
        const int *dim = s->dimH[c];
        for (int k = s->mk0[c]; k < s->mk1[c]; k++)
            for (int j = 0; j < dim[1]; j++)
                for (int i = 0; i < dim[0]; i++) {
                    double ms = s->Ms_s[c][lin(dim, i, j, k)];
                    int64_t q = mlin(s, c, i, j, k);
                    for (int w = 0; w < 3; w++) {
                        double v = ms > 0 ? ms * u[w] : 0.0;
                        s->M[c][w][q] = v;
                        s->M0[c][w][q] = v;
                    }
                }
    }
    return 0;
}

int orc_add_source(orc_sim *s, int comp, int i0, int j0, int k0, int ni, int nj, int nk,
                   const double *table, int64_t n) {
    if (s->nsrc >= 16 || comp < 0 || comp > 2 || !table || n < 0) return -1;
    orc_source *S = &s->src[s->nsrc];
    S->comp = comp;
    S->box[0] = i0; S->box[1] = j0; S->box[2] = k0;
    S->box[3] = ni; S->box[4] = nj; S->box[5] = nk;
    S->table = (double *)malloc((n > 0 ? n : 1) * sizeof(double));
    memcpy(S->table, table, n * sizeof(double));
    S->n = n;
    return s->nsrc++;
}

int orc_add_probe(orc_sim *s, int kind, int field, int i, int j, int k, int film, int64_t cap) {
    if (s->nprobe >= 64 || cap < 1) return -1;
    orc_probe *P = &s->probe[s->nprobe];
    memset(P, 0, sizeof(*P));
    P->kind = kind; P->field = field; P->i = i; P->j = j; P->k = k; P->film = film;
    P->nval = (kind == ORC_PROBE_MEAN_M) ? 3 : 1;
    P->cap = cap;
    P->data = (double *)calloc(cap * P->nval, sizeof(double));
    return s->nprobe++;
}

/* ------------------------------------------------------------------ */
/* discrete curls                                                      */
/* ------------------------------------------------------------------ */

/* (curl E)_c at the H_c site idx: d_{c1} E_{c2} - d_{c2} E_{c1}, forward
 * differences from idx to idx + e_{c1} (resp. e_{c2}).  Out-of-domain
 * neighbours of a non-periodic axis read as zero (they are PEC walls). */
static void curlE_parts(const orc_sim *s, int c, int i, int j, int k, double *d1, double *d2) {
    int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
    int idx[3] = {i, j, k};
    int up1[3] = {i, j, k}, up2[3] = {i, j, k};
    up1[c1] += 1;
    up2[c2] += 1;
    double e2a = at(s, s->E[c2], s->dimE[c2], idx[0], idx[1], idx[2], NULL);
    double e2b = at(s, s->E[c2], s->dimE[c2], up1[0], up1[1], up1[2], NULL);
    double e1a = at(s, s->E[c1], s->dimE[c1], idx[0], idx[1], idx[2], NULL);
    double e1b = at(s, s->E[c1], s->dimE[c1], up2[0], up2[1], up2[2], NULL);
    *d1 = (e2b - e2a) / s->d[c1];
    *d2 = (e1b - e1a) / s->d[c2];
}

/* (curl H)_c at the E_c site idx: backward differences from idx - e_{c1}. */
static void curlH_parts(const orc_sim *s, int c, int i, int j, int k, double *d1, double *d2) {
    int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
    int dn1[3] = {i, j, k}, dn2[3] = {i, j, k};
    dn1[c1] -= 1;
    dn2[c2] -= 1;
    double h2a = at(s, s->H[c2], s->dimH[c2], i, j, k, NULL);
    double h2b = at(s, s->H[c2], s->dimH[c2], dn1[0], dn1[1], dn1[2], NULL);
    double h1a = at(s, s->H[c1], s->dimH[c1], i, j, k, NULL);
    double h1b = at(s, s->H[c1], s->dimH[c1], dn2[0], dn2[1], dn2[2], NULL);
    *d1 = (h2a - h2b) / s->d[c1];
    *d2 = (h1a - h1b) / s->d[c2];
}

static double mag_at(const orc_sim *s, int c, int w, int i, int j, int k) {
    /* M_w at the H_c site (i,j,k) (already folded), 0 if not magnetic */
    if (!s->has_mag || k < s->mk0[c] || k >= s->mk1[c]) return 0.0;
    return s->M[c][w][mlin(s, c, i, j, k)];
}

/* B^ = H + M and B^* = B^ - dt/(2 mu0) curl E at the H_c site (folded
 * indices).  Used for the neighbours of magnetic sites, which are never in
 * a PML, so no psi term enters here. */
static void bhat_site(const orc_sim *s, int c, int i, int j, int k, double *bn, double *bs) {
    double d1, d2;
    curlE_parts(s, c, i, j, k, &d1, &d2);
    double h = s->H[c][lin(s->dimH[c], i, j, k)];
    double b = h + mag_at(s, c, c, i, j, k);
    *bn = b;
    *bs = b - (s->g.dt / (2.0 * ORC_MU0)) * (d1 - d2);
}

/* I_{c'} at the H_c site idx: mean of the <=4 nearest family-c' sites that
 * lie in the domain -- indices {idx_c - 1, idx_c} along c and
 * {idx_c', idx_c' + 1} along c' (reading of where transverse B^ comes from).
 * Pairwise summation. */
static void interp_transverse(const orc_sim *s, int c, int cp, const int *idx, double *In, double *Is) {
    double vn[2][2], vs[2][2];
    int ok[2][2];
    for (int u = 0; u < 2; u++)
        for (int v = 0; v < 2; v++) {
            int q[3] = {idx[0], idx[1], idx[2]};
            q[c] += u - 1;
            q[cp] += v;
            int ii = fold(s, 0, q[0], s->dimH[cp][0]);
            int jj = fold(s, 1, q[1], s->dimH[cp][1]);
            int kk = fold(s, 2, q[2], s->dimH[cp][2]);
            ok[u][v] = (ii >= 0 && jj >= 0 && kk >= 0);
            vn[u][v] = vs[u][v] = 0.0;
            if (ok[u][v]) bhat_site(s, cp, ii, jj, kk, &vn[u][v], &vs[u][v]);
        }
    /* along c' both neighbours are always in the domain (c' integer index
     * idx_c'+1 <= N_c' for a half-integer idx_c'); along c one may be out */
    if (ok[0][0] && ok[1][0]) {
        *In = ((vn[0][0] + vn[1][0]) + (vn[0][1] + vn[1][1])) * 0.25;
        *Is = ((vs[0][0] + vs[1][0]) + (vs[0][1] + vs[1][1])) * 0.25;
    } else if (ok[1][0]) {
        *In = (vn[1][0] + vn[1][1]) * 0.5;
        *Is = (vs[1][0] + vs[1][1]) * 0.5;
    } else {
        *In = (vn[0][0] + vn[0][1]) * 0.5;
        *Is = (vs[0][0] + vs[0][1]) * 0.5;
    }
}

static void cross(const double *a, const double *b, double *r) {
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* eq. (llg_tra4): X = (b + (a.b) a - a x b) / (1 + |a|^2), the solution of
 * X + a x X = b; then the normalisation N(X) = Ms X/|X|. */
static void llg_solve(const double *a, const double *b, double Ms, double *out) {
    double axb[3];
    cross(a, b, axb);
    double ab = dot(a, b), aa = dot(a, a);
    double X[3];
    for (int w = 0; w < 3; w++) X[w] = (b[w] + ab * a[w] - axb[w]) / (1.0 + aa);
    double nx = sqrt(dot(X, X));
    for (int w = 0; w < 3; w++) out[w] = Ms * X[w] / nx;
}

/* ------------------------------------------------------------------ */
/* one H/M half step of length dt/2 using the current E                */
/* ------------------------------------------------------------------ */

/* Returns the number of LLG iterations used (literal mode) or 0. */
static int half_step(orc_sim *s, int literal, double tol, int rmax, int *fail) {
    const double dt = s->g.dt;
    const double kf = ORC_MU0 * dt / 4.0; /* times |gamma|_s: k = mu0 |gamma| dt/4 */
    int r_used = 0;

    /* (1) magnetic sites first (they read pre-step neighbours; Jacobi) */
    if (s->has_mag) {
        for (int c = 0; c < 3; c++) {
            const int *dim = s->dimH[c];
#pragma omp parallel for schedule(static)
            for (int k = s->mk0[c]; k < s->mk1[c]; k++)
                for (int j = 0; j < dim[1]; j++)
                    for (int i = 0; i < dim[0]; i++) {
                        int64_t q = lin(dim, i, j, k);
                        double ms = s->Ms_s[c][q];
                        if (!(ms > 0)) continue;
                        int64_t qm = mlin(s, c, i, j, k);
                        int idx[3] = {i, j, k};
                        double bn, bs;
                        bhat_site(s, c, i, j, k, &bn, &bs);
                        double P[3], Q[3], M[3];
                        P[c] = bs;
                        Q[c] = bn;
                        for (int cp = 0; cp < 3; cp++) {
                            if (cp == c) continue;
                            interp_transverse(s, c, cp, idx, &Q[cp], &P[cp]);
                        }
                        for (int w = 0; w < 3; w++) {
                            P[w] += s->H0[w];
                            Q[w] += s->H0[w];
                            M[w] = s->M[c][w][qm];
                        }
                        double kk = kf * s->ga_s[c][q];
                        double al = s->al_s[c][q];
                        /* eq. (llg_tra6): b = M^n - k (M^n x H_eff^n), H_eff^n = Q - M^n
                         * and M^n x M^n = 0 */
                        double MxQ[3], b[3], a[3], Mn1[3];
                        cross(M, Q, MxQ);
                        for (int w = 0; w < 3; w++) b[w] = M[w] - kk * MxQ[w];
                        if (!literal) {
                            /* eq. (llg_tra5) at the fixed point: H_eff^{n+1} = P - M^{n+1}
                             * and the M^{n+1} part drops out of a x X */
                            for (int w = 0; w < 3; w++) a[w] = -(kk * P[w] + (al / ms) * M[w]);
                            llg_solve(a, b, ms, Mn1);
                        } else {
                            for (int w = 0; w < 3; w++) Mn1[w] = M[w]; /* r = 0 guess */
                        }
                        for (int w = 0; w < 3; w++) s->Mn_tmp[c][w][qm] = Mn1[w];
                        s->Hn_tmp[c][qm] = bs; /* B^* kept; H = B^*_c - M_c below */
                    }
        }
        if (literal) {
            /* the paper's iteration over r: a^{(r)} uses H_eff^{n+1,r-1}
             * = P - M^{n+1,r-1}; stop when max |dM|/Ms < tol over the domain */
            double maxd = 1e300;
            int r = 0;
            while (maxd >= tol) {
                if (r >= rmax) {
                    *fail = 1;
                    break;
                }
                r++;
                maxd = 0.0;
                for (int c = 0; c < 3; c++) {
                    const int *dim = s->dimH[c];
                    for (int k = s->mk0[c]; k < s->mk1[c]; k++)
                        for (int j = 0; j < dim[1]; j++)
                            for (int i = 0; i < dim[0]; i++) {
                                int64_t q = lin(dim, i, j, k);
                                double ms = s->Ms_s[c][q];
                                if (!(ms > 0)) continue;
                                int64_t qm = mlin(s, c, i, j, k);
                                int idx[3] = {i, j, k};
                                double bn, bs;
                                bhat_site(s, c, i, j, k, &bn, &bs);
                                double P[3], Q[3], M[3], Mr[3];
                                P[c] = bs;
                                Q[c] = bn;
                                for (int cp = 0; cp < 3; cp++) {
                                    if (cp == c) continue;
                                    interp_transverse(s, c, cp, idx, &Q[cp], &P[cp]);
                                }
                                for (int w = 0; w < 3; w++) {
                                    P[w] += s->H0[w];
                                    Q[w] += s->H0[w];
                                    M[w] = s->M[c][w][qm];
                                    Mr[w] = s->Mn_tmp[c][w][qm];
                                }
                                double kk = kf * s->ga_s[c][q];
                                double al = s->al_s[c][q];
                                double MxQ[3], b[3], a[3], Mn1[3];
                                cross(M, Q, MxQ);
                                for (int w = 0; w < 3; w++) {
                                    b[w] = M[w] - kk * MxQ[w];
                                    a[w] = -(kk * (P[w] - Mr[w]) + (al / ms) * M[w]);
                                }
                                llg_solve(a, b, ms, Mn1);
                                for (int w = 0; w < 3; w++) {
                                    double dlt = fabs(Mn1[w] - Mr[w]) / ms;
                                    if (dlt > maxd) maxd = dlt;
                                }
                                /* writing in place is safe: a^{(r)} at a site reads only the
                                 * site's own M^{n+1,r-1}; neighbours enter through P and Q,
                                 * which depend on M^n only */
                                s->Hn_tmp[c][qm] = bs;
                                for (int w = 0; w < 3; w++) s->Mn_tmp[c][w][qm] = Mn1[w];
                            }
                }
            }
            r_used = r;
        }
    }

    /* (2) non-magnetic sites: H <- B^* (with CPML psi in the slabs) */
    for (int c = 0; c < 3; c++) {
        int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        const int *dim = s->dimH[c];
        double *pH1 = s->psiH[c][c1], *pH2 = s->psiH[c][c2];
#pragma omp parallel for schedule(static)
        for (int k = 0; k < dim[2]; k++)
            for (int j = 0; j < dim[1]; j++)
                for (int i = 0; i < dim[0]; i++) {
                    int64_t q = lin(dim, i, j, k);
                    if (s->Ms_s[c][q] > 0) continue;
                    int idx[3] = {i, j, k};
                    double d1, d2;
                    curlE_parts(s, c, i, j, k, &d1, &d2);
                    /* H_c sits at half positions along c1 and c2 */
                    if (pH1) {
                        int p = idx[c1];
                        pH1[q] = s->bH[c1][p] * pH1[q] + s->cH[c1][p] * d1;
                        d1 += pH1[q];
                    }
                    if (pH2) {
                        int p = idx[c2];
                        pH2[q] = s->bH[c2][p] * pH2[q] + s->cH[c2][p] * d2;
                        d2 += pH2[q];
                    }
                    /* eq. (iterate_H) with M = 0 */
                    s->H[c][q] = s->H[c][q] - (dt / (2.0 * ORC_MU0)) * (d1 - d2);
                }
    }

    /* (3) commit the magnetic sites: M^{n+1}, and H = B^*_c - M^{n+1}_c
     * (eq. (iterate_H): H^{n+1} = H^n + M^n - M^{n+1} - dt/(2 mu0) curl E) */
    if (s->has_mag) {
        for (int c = 0; c < 3; c++) {
            const int *dim = s->dimH[c];
            for (int k = s->mk0[c]; k < s->mk1[c]; k++)
                for (int j = 0; j < dim[1]; j++)
                    for (int i = 0; i < dim[0]; i++) {
                        int64_t q = lin(dim, i, j, k);
                        if (!(s->Ms_s[c][q] > 0)) continue;
                        int64_t qm = mlin(s, c, i, j, k);
                        for (int w = 0; w < 3; w++) s->M[c][w][qm] = s->Mn_tmp[c][w][qm];
                        s->H[c][q] = s->Hn_tmp[c][qm] - s->M[c][c][qm];
                    }
        }
    }
    return r_used;
}

/* ------------------------------------------------------------------ */
/* E full step                                                         */
/* ------------------------------------------------------------------ */

static double source_value(const orc_sim *s, int c, int i, int j, int k) {
    double J = 0.0;
    for (int n = 0; n < s->nsrc; n++) {
        const orc_source *S = &s->src[n];
        if (S->comp != c) continue;
        if (i < S->box[0] || i >= S->box[0] + S->box[3]) continue;
        if (j < S->box[1] || j >= S->box[1] + S->box[4]) continue;
        if (k < S->box[2] || k >= S->box[2] + S->box[5]) continue;
        /* reading: the table holds J at t_{n+1/2} (time-centred source) */
        if (s->step < S->n) J += S->table[s->step];
    }
    return J;
}

static void e_step(orc_sim *s) {
    for (int c = 0; c < 3; c++) {
        int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        const int *dim = s->dimE[c];
        double *pE1 = s->psiE[c][c1], *pE2 = s->psiE[c][c2];
#pragma omp parallel for schedule(static)
        for (int k = 0; k < dim[2]; k++)
            for (int j = 0; j < dim[1]; j++)
                for (int i = 0; i < dim[0]; i++) {
                    int64_t q = lin(dim, i, j, k);
                    if (s->epec[c][q]) continue;
                    int idx[3] = {i, j, k};
                    double d1, d2;
                    curlH_parts(s, c, i, j, k, &d1, &d2);
                    /* E_c sits at integer positions along c1 and c2 */
                    if (pE1) {
                        int p = idx[c1];
                        pE1[q] = s->bE[c1][p] * pE1[q] + s->cE[c1][p] * d1;
                        d1 += pE1[q];
                    }
                    if (pE2) {
                        int p = idx[c2];
                        pE2[q] = s->bE[c2][p] * pE2[q] + s->cE[c2][p] * d2;
                        d2 += pE2[q];
                    }
                    double J = s->nsrc ? source_value(s, c, i, j, k) : 0.0;
                    s->E[c][q] = s->ca[c][q] * s->E[c][q] + s->cb[c][q] * ((d1 - d2) - J);
                }
    }
}

/* ------------------------------------------------------------------ */
/* probes                                                              */
/* ------------------------------------------------------------------ */

static double film_mean_m(const orc_sim *s, int f, int w) {
    /* sum of M_w over the family-w sites of film f, over its cell count */
    const orc_film *F = &s->film[f];
    const int *dim = s->dimH[w];
    double sum = 0.0;
    int lo[3], hi[3];
    for (int a = 0; a < 3; a++) {
        lo[a] = F->box[a];
        hi[a] = F->box[a] + F->box[3 + a] + (a == w ? 1 : 0);
        if (hi[a] > dim[a]) hi[a] = dim[a];
    }
    for (int k = lo[2]; k < hi[2]; k++)
        for (int j = lo[1]; j < hi[1]; j++)
            for (int i = lo[0]; i < hi[0]; i++) {
                int ii = fold(s, 0, i, dim[0]), jj = fold(s, 1, j, dim[1]), kk = fold(s, 2, k, dim[2]);
                if (ii < 0 || jj < 0 || kk < 0) continue;
                if (!(s->Ms_s[w][lin(dim, ii, jj, kk)] > 0)) continue;
                sum += s->M[w][w][mlin(s, w, ii, jj, kk)];
            }
    return sum / (double)F->ncells;
}

static double film_energy(const orc_sim *s, int f) {
    /* sum over film cells of 1/2 eps0 eps_r sum_c mean_4edges(E_c^2)
     *                     + 1/2 mu0 sum_c mean_2faces(H_c^2), times dV */
    const orc_film *F = &s->film[f];
    double dV = s->d[0] * s->d[1] * s->d[2];
    double W = 0.0;
    for (int k = F->box[2]; k < F->box[2] + F->box[5]; k++)
        for (int j = F->box[1]; j < F->box[1] + F->box[4]; j++)
            for (int i = F->box[0]; i < F->box[0] + F->box[3]; i++) {
                int m = s->id[lin(s->N, i, j, k)];
                if (!(s->mat[m].Ms > 0)) continue;
                int cc[3] = {i, j, k};
                double we = 0.0, wh = 0.0;
                for (int c = 0; c < 3; c++) {
                    int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
                    double e2 = 0.0;
                    for (int u = 0; u < 2; u++)
                        for (int v = 0; v < 2; v++) {
                            int q[3] = {cc[0], cc[1], cc[2]};
                            q[c1] += u;
                            q[c2] += v;
                            double e = at(s, s->E[c], s->dimE[c], q[0], q[1], q[2], NULL);
                            e2 += e * e;
                        }
                    we += e2 / 4.0;
                    double h2 = 0.0;
                    for (int u = 0; u < 2; u++) {
                        int q[3] = {cc[0], cc[1], cc[2]};
                        q[c] += u;
                        double h = at(s, s->H[c], s->dimH[c], q[0], q[1], q[2], NULL);
                        h2 += h * h;
                    }
                    wh += h2 / 2.0;
                }
                W += 0.5 * ORC_EPS0 * s->mat[m].eps_r * we + 0.5 * ORC_MU0 * wh;
            }
    return W * dV;
}

static void record_probes(orc_sim *s) {
    for (int p = 0; p < s->nprobe; p++) {
        orc_probe *P = &s->probe[p];
        double v[3] = {0, 0, 0};
        if (P->kind == ORC_PROBE_FIELD) {
            if (P->field < 3)
                v[0] = at(s, s->E[P->field], s->dimE[P->field], P->i, P->j, P->k, NULL);
            else
                v[0] = at(s, s->H[P->field - 3], s->dimH[P->field - 3], P->i, P->j, P->k, NULL);
        } else if (P->kind == ORC_PROBE_MEAN_M) {
            if (P->film < s->nfilm)
                for (int w = 0; w < 3; w++) v[w] = film_mean_m(s, P->film, w);
        } else if (P->kind == ORC_PROBE_FILM_ENERGY) {
            if (P->film < s->nfilm) v[0] = film_energy(s, P->film);
        }
        int64_t slot = P->n % P->cap;
        for (int w = 0; w < P->nval; w++) P->data[slot * P->nval + w] = v[w];
        P->n++;
    }
}

/* ------------------------------------------------------------------ */
/* time stepping: H/M half step (E^n), E full step, H/M half step      */
/* (E^{n+1}) -- reading of the dt/4 and dt/(2 mu0) factors             */
/* ------------------------------------------------------------------ */

int orc_step(orc_sim *s, int64_t nsteps, int literal, double tol, int rmax) {
    if (!s->have_mat) return 2;
    int fail = 0;
    s->last_r = 0;
    for (int64_t n = 0; n < nsteps; n++) {
        int r1 = half_step(s, literal, tol, rmax, &fail);
        e_step(s);
        int r2 = half_step(s, literal, tol, rmax, &fail);
        if (r1 > s->last_r) s->last_r = r1;
        if (r2 > s->last_r) s->last_r = r2;
        s->step++;
        record_probes(s);
        if (fail) return 3;
    }
    return 0;
}

int orc_last_iterations(const orc_sim *s) { return s->last_r; }

/* ------------------------------------------------------------------ */
/* access                                                              */
/* ------------------------------------------------------------------ */

/* field 0..2 = Ex..Ez, 3..5 = Hx..Hz, 6..8 = M on x/y/z faces (3 comps,
 * component-major), 9..11 = M - M0 on x/y/z faces */
int64_t orc_field_dims(const orc_sim *s, int field, int32_t *dims) {
    const int *d = field < 3 ? s->dimE[field] : s->dimH[(field - 3) % 3];
    dims[0] = d[0]; dims[1] = d[1]; dims[2] = d[2];
    dims[3] = field < 6 ? 1 : 3;
    return (int64_t)d[0] * d[1] * d[2] * dims[3];
}

int orc_get_field(const orc_sim *s, int field, double *dst) {
    if (field < 0 || field > 11) return 1;
    if (field < 3) {
        memcpy(dst, s->E[field], s->nE[field] * sizeof(double));
        return 0;
    }
    if (field < 6) {
        memcpy(dst, s->H[field - 3], s->nH[field - 3] * sizeof(double));
        return 0;
    }
    int c = (field - 6) % 3;
    int delta = field >= 9;
    const int *dim = s->dimH[c];
    int64_t n = s->nH[c];
    memset(dst, 0, 3 * n * sizeof(double));
    if (!s->has_mag) return 0;
    for (int w = 0; w < 3; w++)
        for (int k = s->mk0[c]; k < s->mk1[c]; k++)
            for (int j = 0; j < dim[1]; j++)
                for (int i = 0; i < dim[0]; i++) {
                    int64_t qm = mlin(s, c, i, j, k);
                    double v = s->M[c][w][qm];
                    if (delta) v -= s->M0[c][w][qm];
                    dst[w * n + lin(dim, i, j, k)] = v;
                }
    return 0;
}

int orc_set_field(orc_sim *s, int field, const double *src) {
    if (field < 0 || field > 8) return 1;
    if (field < 3) {
        /* edges that are PEC (walls included) are held at zero */
        for (int64_t q = 0; q < s->nE[field]; q++)
            s->E[field][q] = (s->have_mat && s->epec[field][q]) ? 0.0 : src[q];
        return 0;
    }
    if (field < 6) {
        memcpy(s->H[field - 3], src, s->nH[field - 3] * sizeof(double));
        return 0;
    }
    int c = field - 6;
    const int *dim = s->dimH[c];
    int64_t n = s->nH[c];
    if (!s->has_mag) return 0;
    for (int w = 0; w < 3; w++)
        for (int k = s->mk0[c]; k < s->mk1[c]; k++)
            for (int j = 0; j < dim[1]; j++)
                for (int i = 0; i < dim[0]; i++) {
                    int64_t q = lin(dim, i, j, k);
                    if (!(s->Ms_s[c][q] > 0)) continue;
                    s->M[c][w][mlin(s, c, i, j, k)] = src[w * n + q];
                }
    return 0;
}

int64_t orc_read_probe(const orc_sim *s, int id, double *dst, int64_t cap) {
    if (id < 0 || id >= s->nprobe) return -1;
    const orc_probe *P = &s->probe[id];
    int64_t have = P->n < P->cap ? P->n : P->cap;
    if (cap < have) return -have;
    int64_t first = P->n - have;
    for (int64_t t = 0; t < have; t++) {
        int64_t slot = (first + t) % P->cap;
        for (int w = 0; w < P->nval; w++) dst[t * P->nval + w] = P->data[slot * P->nval + w];
    }
    return have;
}

/* Discrete EM energy at an integer time (design reading of the Yee
 * invariant): W = dV/2 [ sum_e eps_e E_e^2
 *                       + mu0 sum_f (H_f^2 - (dt/(2 mu0))^2 (curl E)_f^2) ]
 * and the Zeeman term W_z = -mu0 dV sum_c sum_{s in family c} H0_c M_{s,c}. */
void orc_energy(const orc_sim *s, double *W_em, double *W_z) {
    double dV = s->d[0] * s->d[1] * s->d[2];
    double we = 0.0, wh = 0.0, wz = 0.0;
    for (int c = 0; c < 3; c++) {
        int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        const int *dim = s->dimE[c];
        for (int k = 0; k < dim[2]; k++)
            for (int j = 0; j < dim[1]; j++)
                for (int i = 0; i < dim[0]; i++) {
                    int64_t q = lin(dim, i, j, k);
                    if (s->epec[c][q]) continue;
                    /* eps_e from cb at sigma = 0: cb = dt/eps_e */
                    int idx[3] = {i, j, k};
                    double se = 0.0;
                    int cnt = 0;
                    for (int u = -1; u <= 0; u++)
                        for (int v = -1; v <= 0; v++) {
                            int cc[3];
                            cc[c] = idx[c];
                            cc[c1] = idx[c1] + u;
                            cc[c2] = idx[c2] + v;
                            int m = cell_id(s, cc[0], cc[1], cc[2]);
                            if (m < 0) continue;
                            se += s->mat[m].eps_r;
                            cnt++;
                        }
                    double eps = ORC_EPS0 * (se / cnt);
                    double e = s->E[c][q];
                    we += eps * e * e;
                }
        const int *dh = s->dimH[c];
        for (int k = 0; k < dh[2]; k++)
            for (int j = 0; j < dh[1]; j++)
                for (int i = 0; i < dh[0]; i++) {
                    double d1, d2;
                    curlE_parts(s, c, i, j, k, &d1, &d2);
                    double cu = (s->g.dt / (2.0 * ORC_MU0)) * (d1 - d2);
                    double h = s->H[c][lin(dh, i, j, k)];
                    wh += h * h - cu * cu;
                }
    }
    if (s->has_mag)
        for (int c = 0; c < 3; c++) {
            const int *dim = s->dimH[c];
            for (int k = s->mk0[c]; k < s->mk1[c]; k++)
                for (int j = 0; j < dim[1]; j++)
                    for (int i = 0; i < dim[0]; i++) {
                        if (!(s->Ms_s[c][lin(dim, i, j, k)] > 0)) continue;
                        /* component c of M at the family-c sites, the part that
                         * enters B = mu0 (H + M) in the H_c update */
                        wz += s->H0[c] * s->M[c][c][mlin(s, c, i, j, k)];
                    }
        }
    *W_em = 0.5 * dV * (we + ORC_MU0 * wh);
    *W_z = -ORC_MU0 * dV * wz;
}

int orc_n_films(const orc_sim *s) { return s->nfilm; }

int orc_film_box(const orc_sim *s, int f, int32_t *box, int64_t *ncells) {
    if (f < 0 || f >= s->nfilm) return 1;
    for (int a = 0; a < 6; a++) box[a] = s->film[f].box[a];
    *ncells = s->film[f].ncells;
    return 0;
}

int64_t orc_step_count(const orc_sim *s) { return s->step; }

void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_get_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
