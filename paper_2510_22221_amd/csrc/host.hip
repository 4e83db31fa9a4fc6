// host.hip -- C ABI of libmpx (include/mpx.h): grid and material setup, film
// discovery, CPML profiles, sources, probes, the step driver (HIP graphs of
// step batches on the handle's stream), field readback and diagnostics.
#include "../../include/mpx.h"
#include "mpx_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <array>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

using namespace mpx;

namespace {

constexpr double PI = 3.14159265358979323846;
constexpr double C0 = 299792458.0;
const double MU0 = 4.0e-7 * PI;
const double EPS0 = 1.0 / (MU0 * C0 * C0);

struct FilmHost {
    int cb[6];      // cell box
    int b0[3], bn[3];
    long long ns;
    long long ncells;
    long long lowest;
    double *M = nullptr, *M1 = nullptr, *H1 = nullptr, *prm = nullptr, *Bn = nullptr, *Bs = nullptr;
    double *Bn2 = nullptr, *Bs2 = nullptr;
    int blk0[3], nblk[3];
    int e0[3], en[3];
    long long nse;
};

struct SrcHost {
    SrcDev dev;
    double *table = nullptr;
};

struct ProbeHost {
    ProbeDev dev;
};

} // namespace

struct mpx_sim {
    mpx_grid_desc g{};
    mpx_precision prec = MPX_F64;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int n[3] = {0, 0, 0};
    int per[3] = {0, 0, 0};
    int px = 0;
    long long nslot = 0;
    double d[3] = {0, 0, 0};
    double dt = 0;
    size_t esz = 8;
    // field buffers: set 0 and its ping-pong partner set 1 (the fused pass
    // reads one set and writes the other); `parity` selects the current one
    void *E[3] = {nullptr, nullptr, nullptr};
    void *H[3] = {nullptr, nullptr, nullptr};
    void *E2[3] = {nullptr, nullptr, nullptr};
    void *H2[3] = {nullptr, nullptr, nullptr};
    int parity = 0;
    int fused = 0; // separate passes (the fastest schedule measured on gfx950)
    int adj_schedule = 0; // mpx_adjoint: 0 tape schedule, 1 plain recompute-per-step schedule, 2 tape schedule
                          // with every half-step transpose in a pass of its own
    // tape schedule: the most device memory the tapes kept from the forward
    // run may take (-1: three quarters of the free memory, with the
    // checkpoints of the other segments; 0: none, every segment recomputed)
    long long adj_resident = -1;
    int kchunk = 16;
    bool narrow = false; // separate passes on 64 x 4 tiles whatever the width (schedule 6)
    void *d_coef = nullptr;
    void *d_coefv = nullptr; // the same rows packed per class (KParams::coefv)
    long long n_coef_ext = 0; // extended triples after the class entries of d_coef
    // materials
    bool have_mat = false;
    std::vector<mpx_material> mats;
    std::vector<uint8_t> ids; // natural cell order
    uint8_t *d_id = nullptr;
    uint8_t *d_cls = nullptr; // per slot: the shared id of the 8 cells around it, or 255
    MatDev *d_mat = nullptr;
    // PML
    int nlo[3] = {0, 0, 0}, nhi[3] = {0, 0, 0};
    void *bE[3] = {}, *cE[3] = {}, *bH[3] = {}, *cH[3] = {};
    void *psiE[3][3] = {}, *psiH[3][3] = {}, *psiE2[3][3] = {};
    bool any_pml = false;
    // films
    std::vector<FilmHost> films;
    FilmDev *d_films = nullptr;
    int4 *d_blocktab = nullptr;
    int4 *d_blocktab_ext = nullptr;
    double *d_partial = nullptr;
    int nblk = 0;
    int nblk_ext = 0;
    double H0[3] = {0, 0, 0};
    double u[3] = {0, 0, 1};
    bool have_u = false;
    // sources, probes
    std::vector<SrcHost> srcs;
    std::vector<ProbeHost> probes;
    ProbeDev *d_probes = nullptr;
    int probe_maxpart = 0; // most partial-sum blocks of an energy probe
    SrcDev *d_srcs = nullptr; // device copy of the source descriptors
    uint8_t *d_pflags = nullptr; // per separate-pass tile: CPML / source / film bits
    uint8_t *d_pflags_w = nullptr; // the same for the wide tiles (when nx >= kWideMinNx)
    int4 *d_mixed = nullptr;     // mixed-class slots without an extended triple (the general path)
    int nmixed = 0;
    uint16_t *d_cls16 = nullptr; // per slot: the class with extended triples (256 + index), 0xffff: mixed list
    long long *d_step = nullptr;
    int *d_flag = nullptr;
    long long step = 0;
    // graphs of step batches, one per starting parity
    int graph_steps = 64;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    hipGraph_t graph[2] = {nullptr, nullptr};
    bool graph_valid[2] = {false, false};
    // with timing on: graphs of the timing_every - 1 untimed steps between
    // two timed ones, per starting parity, and the parity each ends at
    hipGraphExec_t tgexec[2] = {nullptr, nullptr};
    hipGraph_t tgraph[2] = {nullptr, nullptr};
    bool tgraph_valid[2] = {false, false};
    int tgraph_end[2] = {0, 0};
    // timing
    int timing_every = 0;
    std::vector<hipEvent_t> ev;
    size_t evi = 0;
    double t_ms[3] = {0, 0, 0};
    long long t_n[3] = {0, 0, 0};
    // errors
    bool dead = false;
    std::string err;
};

namespace {

mpx_status fail(mpx_sim *s, mpx_status st, const std::string &msg) {
    if (s) s->err = msg;
    return st;
}

mpx_status dev_fail(mpx_sim *s, hipError_t e, const char *what) {
    s->dead = true;
    s->err = std::string(what) + ": " + hipGetErrorString(e);
    return MPX_E_DEVICE;
}

#define CK(call)                                                   \
    do {                                                           \
        hipError_t _e = (call);                                    \
        if (_e != hipSuccess) return dev_fail(s, _e, #call);       \
    } while (0)

long long natural_dim(const mpx_sim *s, int field, int a) {
    // E_c: N_c along c; H_c: N_c (+1 if not periodic) along c; the
    // other axes the reverse
    const int c = field % 3;
    const bool is_e = field < 3;
    const bool half = is_e ? (a == c) : (a != c);
    return half ? s->n[a] : s->n[a] + (s->per[a] ? 0 : 1);
}

int fold_h(int i, int n, int per) {
    if (per) {
        if (i < 0) i += n;
        if (i >= n) i -= n;
        return i;
    }
    return (i < 0 || i >= n) ? -1 : i;
}

int cell_id_h(const mpx_sim *s, int i, int j, int k) {
    int ii = fold_h(i, s->n[0], s->per[0]), jj = fold_h(j, s->n[1], s->per[1]), kk = fold_h(k, s->n[2], s->per[2]);
    if (ii < 0 || jj < 0 || kk < 0) return -1;
    return s->ids[(size_t)ii + (size_t)s->n[0] * ((size_t)jj + (size_t)s->n[1] * kk)];
}

// Ms, alpha, |gamma| of the face of family c at natural index idx (the mean
// over the two cells sharing it, alpha and gamma over the magnetic ones)
void site_params_h(const mpx_sim *s, int c, const int *idx, double &ms, double &al, double &ga) {
    double sm = 0, sa = 0, sg = 0;
    int cnt = 0, nm = 0;
    for (int u = -1; u <= 0; u++) {
        int cc[3] = {idx[0], idx[1], idx[2]};
        cc[c] += u;
        int m = cell_id_h(s, cc[0], cc[1], cc[2]);
        if (m < 0) continue;
        cnt++;
        sm += s->mats[m].Ms;
        if (s->mats[m].Ms > 0) {
            nm++;
            sa += s->mats[m].alpha;
            sg += s->mats[m].gamma_abs;
        }
    }
    ms = cnt ? sm / cnt : 0.0;
    al = nm ? sa / nm : 0.0;
    ga = nm ? sg / nm : 0.0;
}

bool edge_is_pec_h(const mpx_sim *s, int c, const int *idx) {
    const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
    for (int a : {c1, c2})
        if (!s->per[a] && (idx[a] == 0 || idx[a] >= s->n[a])) return true;
    for (int u = -1; u <= 0; u++)
        for (int v = -1; v <= 0; v++) {
            int cc[3];
            cc[c] = idx[c];
            cc[c1] = idx[c1] + u;
            cc[c2] = idx[c2] + v;
            int m = cell_id_h(s, cc[0], cc[1], cc[2]);
            if (m >= 0 && s->mats[m].is_pec) return true;
        }
    return false;
}

bool in_pml_cell(const mpx_sim *s, int a, int i) { return i < s->nlo[a] || i >= s->n[a] - s->nhi[a]; }

// buffer sets by parity
void *const *Eset(const mpx_sim *s, int par) { return par ? s->E2 : s->E; }
void *const *Hset(const mpx_sim *s, int par) { return par ? s->H2 : s->H; }
void *psiEset(const mpx_sim *s, int par, int c, int w) { return par ? s->psiE2[c][w] : s->psiE[c][w]; }

enum ParamMode { MODE_INPLACE = 0, MODE_FUSED = 1, MODE_AFTER_FUSED = 2 };

template <typename T>
void fill_params(const mpx_sim *s, KParams<T> &p, int mode = MODE_INPLACE, int par = -1) {
    memset(&p, 0, sizeof(p));
    if (par < 0) par = s->parity;
    for (int a = 0; a < 3; a++) {
        p.n[a] = s->n[a];
        p.per[a] = s->per[a];
        p.d[a] = s->d[a];
        p.dT[a] = (T)s->d[a];
        p.invd[a] = (T)(1.0 / s->d[a]);
        p.nlo[a] = s->nlo[a];
        p.nhi[a] = s->nhi[a];
        p.bE[a] = (const T *)s->bE[a];
        p.cE[a] = (const T *)s->cE[a];
        p.bH[a] = (const T *)s->bH[a];
        p.cH[a] = (const T *)s->cH[a];
        const int nx = par ^ 1;
        p.E[a] = (T *)Eset(s, mode == MODE_AFTER_FUSED ? nx : par)[a];
        p.H[a] = (T *)Hset(s, par)[a];
        p.Hw[a] = (T *)Hset(s, mode == MODE_AFTER_FUSED ? nx : par)[a];
        p.Eb[a] = (T *)Eset(s, nx)[a];
        p.Hb[a] = (T *)Hset(s, nx)[a];
        p.H0[a] = s->H0[a];
        for (int w = 0; w < 3; w++) {
            p.psiE[a][w] = (T *)psiEset(s, par, a, w);
            p.psiEb[a][w] = (T *)psiEset(s, nx, a, w);
            p.psiH[a][w] = (T *)s->psiH[a][w];
        }
    }
    p.px = s->px;
    p.hcd = s->dt / (2.0 * MU0);
    p.hc = (T)p.hcd;
    p.dt = s->dt;
    p.inv_dt = 1.0 / s->dt;
    p.eps0 = EPS0;
    p.mu0 = MU0;
    p.kf = MU0 * s->dt / 4.0;
    p.dV = s->d[0] * s->d[1] * s->d[2];
    p.id = s->d_id;
    p.cls = s->d_cls;
    p.mat = s->d_mat;
    p.coef = (const CoefDev<T> *)s->d_coef;
    p.coefx = p.coef + kCoefEntries;
    p.coefv = (const T *)s->d_coefv;
    p.nfilm = (int)s->films.size();
    p.films = s->d_films;
    p.blocktab = s->d_blocktab;
    p.blocktab_ext = s->d_blocktab_ext;
    p.nblk_ext = s->nblk_ext;
    p.partial = s->d_partial;
    p.nsrc = (int)s->srcs.size();
    for (int i = 0; i < p.nsrc; i++) p.src[i] = s->srcs[i].dev;
    p.srcs = s->d_srcs;
    p.pflags = s->d_pflags;
    p.pflags_w = s->d_pflags_w;
    p.wide = s->d_pflags_w != nullptr && !s->narrow;
    p.mixed = s->d_mixed;
    p.nmixed = s->nmixed;
    p.cls16 = s->d_cls16;
    p.probes = s->d_probes;
    p.step = s->d_step;
    p.flag = s->d_flag;
}

void free_films(mpx_sim *s) {
    for (auto &f : s->films) {
        (void)hipFree(f.M);
        (void)hipFree(f.M1);
        (void)hipFree(f.H1);
        (void)hipFree(f.prm);
        (void)hipFree(f.Bn);
        (void)hipFree(f.Bs);
        (void)hipFree(f.Bn2);
        (void)hipFree(f.Bs2);
    }
    s->films.clear();
    (void)hipFree(s->d_films);
    (void)hipFree(s->d_blocktab);
    (void)hipFree(s->d_blocktab_ext);
    (void)hipFree(s->d_partial);
    s->d_films = nullptr;
    s->d_blocktab = nullptr;
    s->d_blocktab_ext = nullptr;
    s->d_partial = nullptr;
    s->nblk = 0;
    s->nblk_ext = 0;
}

void drop_graph(mpx_sim *s) {
    for (int q = 0; q < 2; q++) {
        if (s->gexec[q]) (void)hipGraphExecDestroy(s->gexec[q]);
        if (s->graph[q]) (void)hipGraphDestroy(s->graph[q]);
        s->gexec[q] = nullptr;
        s->graph[q] = nullptr;
        s->graph_valid[q] = false;
        if (s->tgexec[q]) (void)hipGraphExecDestroy(s->tgexec[q]);
        if (s->tgraph[q]) (void)hipGraphDestroy(s->tgraph[q]);
        s->tgexec[q] = nullptr;
        s->tgraph[q] = nullptr;
        s->tgraph_valid[q] = false;
    }
}

// connected components of magnetic cells -> bounding boxes; boxes closer than
// two cells on every axis are merged; ordered by lowest linear cell index
std::vector<FilmHost> discover_films(const mpx_sim *s) {
    const long long ncell = (long long)s->n[0] * s->n[1] * s->n[2];
    std::vector<int> lab(ncell, -1);
    std::vector<long long> stack;
    struct Box {
        int lo[3], hi[3];
        long long low;
    };
    std::vector<Box> boxes;
    for (long long q = 0; q < ncell; q++) {
        if (lab[q] >= 0 || !(s->mats[s->ids[q]].Ms > 0)) continue;
        Box b{{1 << 30, 1 << 30, 1 << 30}, {-1, -1, -1}, q};
        stack.clear();
        stack.push_back(q);
        lab[q] = (int)boxes.size();
        while (!stack.empty()) {
            long long pq = stack.back();
            stack.pop_back();
            int c[3] = {(int)(pq % s->n[0]), (int)((pq / s->n[0]) % s->n[1]), (int)(pq / ((long long)s->n[0] * s->n[1]))};
            for (int a = 0; a < 3; a++) {
                b.lo[a] = std::min(b.lo[a], c[a]);
                b.hi[a] = std::max(b.hi[a], c[a] + 1);
            }
            for (int a = 0; a < 3; a++)
                for (int sg = -1; sg <= 1; sg += 2) {
                    int nc[3] = {c[0], c[1], c[2]};
                    nc[a] += sg;
                    if (nc[a] < 0 || nc[a] >= s->n[a]) continue;
                    long long pn = nc[0] + (long long)s->n[0] * (nc[1] + (long long)s->n[1] * nc[2]);
                    if (lab[pn] < 0 && s->mats[s->ids[pn]].Ms > 0) {
                        lab[pn] = (int)boxes.size();
                        stack.push_back(pn);
                    }
                }
        }
        boxes.push_back(b);
    }
    bool merged = true;
    while (merged) {
        merged = false;
        for (size_t x = 0; x < boxes.size() && !merged; x++)
            for (size_t y = x + 1; y < boxes.size() && !merged; y++) {
                bool close = true;
                for (int a = 0; a < 3; a++) {
                    int gap = boxes[y].lo[a] >= boxes[x].hi[a]   ? boxes[y].lo[a] - boxes[x].hi[a]
                              : boxes[x].lo[a] >= boxes[y].hi[a] ? boxes[x].lo[a] - boxes[y].hi[a]
                                                                 : 0;
                    if (gap >= 2) close = false;
                }
                if (close) {
                    for (int a = 0; a < 3; a++) {
                        boxes[x].lo[a] = std::min(boxes[x].lo[a], boxes[y].lo[a]);
                        boxes[x].hi[a] = std::max(boxes[x].hi[a], boxes[y].hi[a]);
                    }
                    boxes[x].low = std::min(boxes[x].low, boxes[y].low);
                    boxes.erase(boxes.begin() + y);
                    merged = true;
                }
            }
    }
    std::sort(boxes.begin(), boxes.end(), [](const Box &a, const Box &b) { return a.low < b.low; });
    std::vector<FilmHost> out;
    for (auto &b : boxes) {
        FilmHost f{};
        for (int a = 0; a < 3; a++) {
            f.cb[a] = b.lo[a];
            f.cb[3 + a] = b.hi[a] - b.lo[a];
        }
        f.lowest = b.low;
        f.ncells = 0;
        for (int k = b.lo[2]; k < b.hi[2]; k++)
            for (int j = b.lo[1]; j < b.hi[1]; j++)
                for (int i = b.lo[0]; i < b.hi[0]; i++)
                    if (s->mats[s->ids[i + (size_t)s->n[0] * (j + (size_t)s->n[1] * k)]].Ms > 0) f.ncells++;
        out.push_back(f);
    }
    return out;
}

template <typename T>
mpx_status upload_profiles(mpx_sim *s) {
    const double m = s->g.pml_order > 0 ? s->g.pml_order : 3.0;
    const double f = s->g.pml_sigma_factor > 0 ? s->g.pml_sigma_factor : 0.8;
    const double eta0 = std::sqrt(MU0 / EPS0);
    for (int a = 0; a < 3; a++) {
        const int n = s->n[a];
        const int nlo = s->nlo[a], nhi = s->nhi[a];
        if (nlo == 0 && nhi == 0) continue;
        std::vector<T> be(n + 1), ce(n + 1), bh(n + 1), ch(n + 1);
        const double smax = f * (m + 1.0) / (eta0 * s->d[a]);
        for (int pp = 0; pp <= n; pp++)
            for (int half = 0; half < 2; half++) {
                const double x = pp + 0.5 * half;
                double rho = 0.0;
                if (nlo > 0 && x < nlo) rho = (nlo - x) / nlo;
                if (nhi > 0 && x > n - nhi) rho = (x - (n - nhi)) / nhi;
                const double sig = smax * std::pow(rho, m);
                if (half == 0) {
                    const double b = std::exp(-sig * s->dt / EPS0);
                    be[pp] = (T)b;
                    ce[pp] = (T)(b - 1.0);
                } else {
                    const double b = std::exp(-sig * (0.5 * s->dt) / EPS0);
                    bh[pp] = (T)b;
                    ch[pp] = (T)(b - 1.0);
                }
            }
        void **dst[4] = {&s->bE[a], &s->cE[a], &s->bH[a], &s->cH[a]};
        std::vector<T> *src[4] = {&be, &ce, &bh, &ch};
        for (int q = 0; q < 4; q++) {
            CK(hipMalloc(dst[q], (n + 1) * sizeof(T)));
            CK(hipMemcpy(*dst[q], src[q]->data(), (n + 1) * sizeof(T), hipMemcpyHostToDevice));
        }
        const int S = nlo + nhi;
        size_t cnt = a == 0 ? (size_t)S * s->n[1] * s->n[2]
                     : a == 1 ? (size_t)s->px * S * s->n[2]
                              : (size_t)s->px * s->n[1] * S;
        for (int c = 0; c < 3; c++) {
            if (c == a) continue;
            CK(hipMalloc(&s->psiE[c][a], cnt * sizeof(T)));
            CK(hipMalloc(&s->psiE2[c][a], cnt * sizeof(T)));
            CK(hipMalloc(&s->psiH[c][a], cnt * sizeof(T)));
            CK(hipMemset(s->psiE[c][a], 0, cnt * sizeof(T)));
            CK(hipMemset(s->psiE2[c][a], 0, cnt * sizeof(T)));
            CK(hipMemset(s->psiH[c][a], 0, cnt * sizeof(T)));
        }
    }
    return MPX_OK;
}

// the number of probes that ride in the merged H/M launch: all of them when
// every one reads only E or a film's mean-M partials and the launch has film
// blocks on 256 x 1 tiles, else none (the probe launch takes them)
int folded_probes(const mpx_sim *s, bool wide) {
    const int np = (int)s->probes.size();
    if (np == 0 || s->nblk == 0 || !wide) return 0;
    for (const ProbeHost &pr : s->probes)
        if (!probe_reads_e_or_m(pr.dev.kind, pr.dev.field)) return 0;
    return np;
}

// One step of the body (not the last): the fused pass or the two separate
// stencil passes, then the film half steps and the probes.  `par` is the
// current buffer parity; the fused schedule flips it.
template <typename T>
mpx_status run_body(mpx_sim *s, int &par, bool timed) {
    const int nblk = s->nblk;
    const int np = (int)s->probes.size();
    hipStream_t st = s->stream;
    // six events per timed step: group g (0 = main stencil kernel, 1 = second
    // stencil kernel of the two-pass schedule, 2 = film and probe kernels)
    // brackets with slots base + 2g and base + 2g + 1
    size_t base = s->evi;
    if (timed) {
        while (s->ev.size() < base + 6) {
            hipEvent_t e;
            CK(hipEventCreate(&e));
            s->ev.push_back(e);
        }
        s->evi += 6;
    }
    auto rec = [&](int g, int end) -> mpx_status {
        if (timed) CK(hipEventRecord(s->ev[base + 2 * g + end], st));
        return MPX_OK;
    };
    mpx_status r;
    if (s->fused) {
        KParams<T> pa, pb;
        fill_params<T>(s, pa, MODE_FUSED, par);
        fill_params<T>(s, pb, MODE_AFTER_FUSED, par);
        if ((r = rec(0, 0)) != MPX_OK) return r;
        if (s->fused == 1)
            CK(launch_sweep<T>(pa, s->kchunk, st));
        else
            CK(launch_fused<T>(pa, s->kchunk, s->fused - 1, st));
        if ((r = rec(0, 1)) != MPX_OK) return r;
        if ((r = rec(1, 0)) != MPX_OK) return r; // no second stencil kernel
        if ((r = rec(1, 1)) != MPX_OK) return r;
        if ((r = rec(2, 0)) != MPX_OK) return r;
        CK(launch_film<T>(pb, nblk, 1, 0, st));
        CK(launch_probes<T>(pb, np, s->probe_maxpart, st));
        if (nblk)
            CK(launch_film<T>(pb, nblk, 2, 1, st));
        else
            CK(launch_tick(s->d_step, st));
        if ((r = rec(2, 1)) != MPX_OK) return r;
        par ^= 1;
        return MPX_OK;
    }
    // two-pass schedule, in place: E pass, the film's first half step (its
    // prepass reads H before the bulk pass moves it) and probes, then the
    // film's second half step with the bulk H pass (and the probes, when all
    // of them read only E or mean M: the H/M launch writes neither)
    KParams<T> p;
    fill_params<T>(s, p, MODE_INPLACE, par);
    const int npf = folded_probes(s, p.wide != 0);
    if ((r = rec(0, 0)) != MPX_OK) return r;
    CK(launch_epass<T>(p, st));
    if ((r = rec(0, 1)) != MPX_OK) return r;
    if ((r = rec(2, 0)) != MPX_OK) return r;
    CK(launch_film<T>(p, nblk, 1, 0, st));
    if (npf == 0) CK(launch_probes<T>(p, np, s->probe_maxpart, st));
    if ((r = rec(2, 1)) != MPX_OK) return r;
    if ((r = rec(1, 0)) != MPX_OK) return r;
    CK(launch_hbulk_film<T>(p, nblk, 1, st, npf));
    if ((r = rec(1, 1)) != MPX_OK) return r;
    return MPX_OK;
}

// the last step of a call: E pass, first H/M half step (probes), commit
template <typename T>
mpx_status run_last(mpx_sim *s, int par, hipStream_t st = nullptr) {
    KParams<T> p;
    fill_params<T>(s, p, MODE_INPLACE, par);
    if (!st) st = s->stream;
    CK(launch_epass<T>(p, st));
    CK(launch_film<T>(p, s->nblk, 1, 0, st));
    CK(launch_probes<T>(p, (int)s->probes.size(), s->probe_maxpart, st));
    CK(launch_commit<T>(p, s->nblk, st));
    CK(launch_hbulk<T>(p, 1, 1, st));
    return MPX_OK;
}

template <typename T>
mpx_status enqueue_steps(mpx_sim *s, long long nsteps) {
    hipStream_t st = s->stream;
    const int nblk = s->nblk;
    {
        // bracket: first H/M half step with E^n, in place
        KParams<T> p;
        fill_params<T>(s, p, MODE_INPLACE, s->parity);
        CK(launch_film<T>(p, nblk, 1, 0, st));
        CK(launch_commit<T>(p, nblk, st));
        CK(launch_hbulk<T>(p, 1, 0, st));
    }
    long long body = nsteps - 1;
    mpx_status r;
    int par = s->parity;
    if (s->timing_every > 0) {
        // every timing_every-th step timed with events (direct launches);
        // the untimed runs between them replayed from a captured graph
        // unless graphs are off
        s->evi = 0;
        const int U = s->timing_every - 1;
        long long n = 0;
        while (n < body) {
            if ((r = run_body<T>(s, par, true)) != MPX_OK) return r;
            n++;
            if (U > 0 && s->graph_steps > 0 && body - n >= U) {
                if (!s->tgraph_valid[par]) {
                    CK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                    int cp = par;
                    for (int u = 0; u < U; u++) {
                        r = run_body<T>(s, cp, false);
                        if (r != MPX_OK) {
                            hipGraph_t g;
                            (void)hipStreamEndCapture(st, &g);
                            return r;
                        }
                    }
                    CK(hipStreamEndCapture(st, &s->tgraph[par]));
                    CK(hipGraphInstantiate(&s->tgexec[par], s->tgraph[par], nullptr, nullptr, 0));
                    s->tgraph_valid[par] = true;
                    s->tgraph_end[par] = cp;
                }
                CK(hipGraphLaunch(s->tgexec[par], st));
                par = s->tgraph_end[par];
                n += U;
            } else {
                for (; n < body && (n % s->timing_every) != 0; n++)
                    if ((r = run_body<T>(s, par, false)) != MPX_OK) return r;
            }
        }
        if ((r = run_last<T>(s, par)) != MPX_OK) return r;
        s->parity = par;
        CK(hipStreamSynchronize(st));
        for (int g = 0; g < 3; g++) {
            s->t_ms[g] = 0;
            s->t_n[g] = 0;
        }
        for (size_t q = 0; q + 5 < s->evi; q += 6)
            for (int g = 0; g < 3; g++) {
                float a = 0;
                CK(hipEventElapsedTime(&a, s->ev[q + 2 * g], s->ev[q + 2 * g + 1]));
                s->t_ms[g] += a;
                s->t_n[g]++;
            }
        if (s->fused) s->t_n[1] = 0;
        return MPX_OK;
    }
    // HIP graph of G body steps (G even, so the buffer parity is unchanged
    // after a replay); one graph per starting parity
    const int G = (s->graph_steps + 1) / 2 * 2;
    if (G > 0 && body >= G) {
        if (!s->graph_valid[par]) {
            CK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            int cp = par;
            for (int n = 0; n < G; n++) {
                r = run_body<T>(s, cp, false);
                if (r != MPX_OK) {
                    hipGraph_t g;
                    (void)hipStreamEndCapture(st, &g);
                    return r;
                }
            }
            CK(hipStreamEndCapture(st, &s->graph[par]));
            CK(hipGraphInstantiate(&s->gexec[par], s->graph[par], nullptr, nullptr, 0));
            s->graph_valid[par] = true;
        }
        while (body >= G) {
            CK(hipGraphLaunch(s->gexec[par], st));
            body -= G;
        }
    }
    for (long long n = 0; n < body; n++)
        if ((r = run_body<T>(s, par, false)) != MPX_OK) return r;
    r = run_last<T>(s, par);
    s->parity = par;
    return r;
}

mpx_status check_live(mpx_sim *s) {
    if (!s) return MPX_E_INVALID;
    if (s->dead) return MPX_E_DEVICE;
    hipError_t e = hipSetDevice(s->device);
    if (e != hipSuccess) return dev_fail(s, e, "hipSetDevice");
    return MPX_OK;
}

// per-tile flags of the separate passes (tx x ty slots of one plane, with a
// one-slot halo): 1 = touches a CPML slab, 8 = a y or z CPML slab (1 without
// 8: x slabs only), 2 = a source box, 4 = a film's face box; with a periodic axis every tile may see index 0 through the wrap
std::vector<uint8_t> tile_flags(const mpx_sim *s, int tx, int ty) {
    const int nxt = (s->n[0] + tx - 1) / tx, nyt = (s->n[1] + ty - 1) / ty;
    const int nt = nxt * nyt * s->n[2];
    std::vector<uint8_t> fl(nt, 0);
    const bool wrap = s->per[0] || s->per[1] || s->per[2];
    for (int t = 0; t < nt; t++) {
        const int i0 = (t % nxt) * tx, j0 = ((t / nxt) % nyt) * ty, k = t / (nxt * nyt);
        const int lo[3] = {i0 - 1, j0 - 1, k - 1}, hi[3] = {i0 + tx, j0 + ty, k + 1};
        uint8_t f = 0;
        for (int a = 0; a < 3; a++) {
            const bool slab = (s->nlo[a] > 0 && lo[a] < s->nlo[a]) || (s->nhi[a] > 0 && hi[a] >= s->n[a] - s->nhi[a]);
            if (slab) f |= a == 0 ? 1 : 1 | 8;
        }
        for (auto &src : s->srcs) {
            bool in = true;
            for (int a = 0; a < 3; a++)
                if (src.dev.box[a] + src.dev.box[3 + a] <= lo[a] || src.dev.box[a] > hi[a]) in = false;
            if (in || wrap) f |= 2;
        }
        for (auto &fm : s->films) {
            bool in = true;
            for (int a = 0; a < 3; a++)
                if (fm.b0[a] + fm.bn[a] <= lo[a] || fm.b0[a] > hi[a]) in = false;
            if (in || wrap) f |= 4;
        }
        fl[t] = f;
    }
    return fl;
}

mpx_status update_pass_flags(mpx_sim *s) {
    const std::vector<uint8_t> fl = tile_flags(s, kPassTX, kPassTY);
    (void)hipFree(s->d_pflags);
    s->d_pflags = nullptr;
    // rounded up to whole 4-byte words: the E pass reads its flag byte
    // through the scalar cache, one aligned word at a time
    CK(hipMalloc(&s->d_pflags, (fl.size() + 4) / 4 * 4));
    CK(hipMemcpy(s->d_pflags, fl.data(), fl.size(), hipMemcpyHostToDevice));
    (void)hipFree(s->d_pflags_w);
    s->d_pflags_w = nullptr;
    if (s->n[0] >= kWideMinNx) {
        const std::vector<uint8_t> fw = tile_flags(s, kWideTX, kWideTY);
        CK(hipMalloc(&s->d_pflags_w, (fw.size() + 4) / 4 * 4));
        CK(hipMemcpy(s->d_pflags_w, fw.data(), fw.size(), hipMemcpyHostToDevice));
    }
    return MPX_OK;
}

mpx_status upload_probes(mpx_sim *s) {
    (void)hipFree(s->d_probes);
    s->d_probes = nullptr;
    s->probe_maxpart = 0;
    for (auto &pr : s->probes) s->probe_maxpart = std::max<int>(s->probe_maxpart, (int)pr.dev.npart);
    if (s->probes.empty()) return MPX_OK;
    std::vector<ProbeDev> v;
    for (auto &pr : s->probes) v.push_back(pr.dev);
    CK(hipMalloc(&s->d_probes, v.size() * sizeof(ProbeDev)));
    CK(hipMemcpy(s->d_probes, v.data(), v.size() * sizeof(ProbeDev), hipMemcpyHostToDevice));
    return MPX_OK;
}

} // namespace

// ===========================================================================
// Batched stepping of several simulations
// ===========================================================================
struct mpx_batch {
    std::vector<mpx_sim *> sims;
    mpx_precision prec = MPX_F64;
    int device = 0;
    hipStream_t stream = nullptr;
    int variant = 1, kchunk = 16;
    size_t psize = 0;
    void *d_pa[2] = {nullptr, nullptr}; // fused-pass parameters, flip 0 / 1
    void *d_pb[2] = {nullptr, nullptr}; // film / probe parameters after it
    int4 *d_work = nullptr; // fused variants: (instance, tile, z-chunk)
    int nwork = 0;
    int4 *d_work2 = nullptr; // separate passes: (instance, x tile, y tile, plane)
    int nwork2 = 0;
    int2 *d_wmixed = nullptr; // mixed-slot blocks: (instance, first entry)
    int nwmixed = 0;
    bool any_xcls = false; // a member has extended-table slots
    int2 *d_wfilm = nullptr, *d_wext = nullptr, *d_wprobe = nullptr;
    int nwfilm = 0, nwext = 0, nwprobe = 0;
    int probe_maxpart = 0;
    int *d_tick = nullptr;
    int ntick = 0;
    int graph_steps = 64;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    bool graph_valid = false;
    std::vector<hipEvent_t> ev;
    std::string err;
    bool dead = false;
};

namespace {

mpx_status bdev_fail(mpx_batch *b, hipError_t e, const char *what) {
    b->dead = true;
    b->err = std::string(what) + ": " + hipGetErrorString(e);
    return MPX_E_DEVICE;
}

#define BCK(call)                                                  \
    do {                                                           \
        hipError_t _e = (call);                                    \
        if (_e != hipSuccess) return bdev_fail(b, _e, #call);      \
    } while (0)

void batch_drop_graph(mpx_batch *b) {
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
    b->graph_valid = false;
}

template <typename T>
mpx_status batch_tables(mpx_batch *b) {
    b->any_xcls = false;
    // tiles instance by instance, in the single-instance order
    std::vector<int4> work, work2;
    std::vector<int2> wmixed, wfilm, wext, wprobe;
    std::vector<int> tick;
    for (int q = 0; q < (int)b->sims.size(); q++) {
        const mpx_sim *s = b->sims[q];
        if (b->variant == 0) {
            const int nxt = (s->n[0] + kPassTX - 1) / kPassTX, nyt = (s->n[1] + kPassTY - 1) / kPassTY;
            for (int k = 0; k < s->n[2]; k++)
                for (int by = 0; by < nyt; by++)
                    for (int bx = 0; bx < nxt; bx++) work2.push_back(make_int4(q, bx, by, k));
            for (int m = 0; m < s->nmixed; m += 256) wmixed.push_back(make_int2(q, m));
            if (s->d_cls16) b->any_xcls = true;
        } else {
            // tiles of 64 x 4 columns (register sweep) or 64 x 8 (LDS-staged)
            const int nxt = (s->n[0] + 63) / 64, nyt = b->variant == 1 ? (s->n[1] + 3) / 4 : (s->n[1] + 7) / 8;
            const int nzc = (s->n[2] + b->kchunk - 1) / b->kchunk;
            for (int t = 0; t < nxt * nyt * nzc; t++) work.push_back(make_int4(q, t, b->kchunk, 0));
        }
        for (int k = 0; k < s->nblk; k++) wfilm.push_back(make_int2(q, k));
        for (int k = 0; k < s->nblk_ext; k++) wext.push_back(make_int2(q, k));
        for (int k = 0; k < (int)s->probes.size(); k++) wprobe.push_back(make_int2(q, k));
        if (s->nblk == 0) tick.push_back(q);
    }
    b->probe_maxpart = 0;
    for (const mpx_sim *s : b->sims) b->probe_maxpart = std::max(b->probe_maxpart, s->probe_maxpart);
    (void)hipFree(b->d_work);
    (void)hipFree(b->d_work2);
    (void)hipFree(b->d_wmixed);
    (void)hipFree(b->d_wfilm);
    (void)hipFree(b->d_wext);
    (void)hipFree(b->d_wprobe);
    (void)hipFree(b->d_tick);
    b->d_work = nullptr;
    b->d_work2 = nullptr;
    b->d_wmixed = nullptr;
    b->d_wfilm = b->d_wext = b->d_wprobe = nullptr;
    b->d_tick = nullptr;
    b->nwork = (int)work.size();
    b->nwork2 = (int)work2.size();
    b->nwmixed = (int)wmixed.size();
    b->nwfilm = (int)wfilm.size();
    b->nwext = (int)wext.size();
    b->nwprobe = (int)wprobe.size();
    b->ntick = (int)tick.size();
    BCK(hipMalloc(&b->d_work, std::max<size_t>(1, work.size()) * sizeof(int4)));
    if (!work.empty()) BCK(hipMemcpy(b->d_work, work.data(), work.size() * sizeof(int4), hipMemcpyHostToDevice));
    BCK(hipMalloc(&b->d_work2, std::max<size_t>(1, work2.size()) * sizeof(int4)));
    if (!work2.empty())
        BCK(hipMemcpy(b->d_work2, work2.data(), work2.size() * sizeof(int4), hipMemcpyHostToDevice));
    auto up2 = [&](int2 **d, std::vector<int2> &v) -> mpx_status {
        BCK(hipMalloc(d, std::max<size_t>(1, v.size()) * sizeof(int2)));
        if (!v.empty()) BCK(hipMemcpy(*d, v.data(), v.size() * sizeof(int2), hipMemcpyHostToDevice));
        return MPX_OK;
    };
    mpx_status r;
    if ((r = up2(&b->d_wmixed, wmixed)) != MPX_OK) return r;
    if ((r = up2(&b->d_wfilm, wfilm)) != MPX_OK) return r;
    if ((r = up2(&b->d_wext, wext)) != MPX_OK) return r;
    if ((r = up2(&b->d_wprobe, wprobe)) != MPX_OK) return r;
    BCK(hipMalloc(&b->d_tick, std::max<size_t>(1, tick.size()) * sizeof(int)));
    if (!tick.empty()) BCK(hipMemcpy(b->d_tick, tick.data(), tick.size() * sizeof(int), hipMemcpyHostToDevice));
    return MPX_OK;
}

// the instances' parameters at their current parity (flip 0) and flipped;
// the separate passes work in place (flip 0 only)
template <typename T>
mpx_status batch_params(mpx_batch *b) {
    const size_t n = b->sims.size();
    std::vector<KParams<T>> pa(n), pb(n);
    for (int f = 0; f < 2; f++) {
        for (size_t q = 0; q < n; q++) {
            const mpx_sim *s = b->sims[q];
            if (b->variant == 0) {
                fill_params<T>(s, pa[q], MODE_INPLACE, s->parity);
                pb[q] = pa[q];
            } else {
                fill_params<T>(s, pa[q], MODE_FUSED, s->parity ^ f);
                fill_params<T>(s, pb[q], MODE_AFTER_FUSED, s->parity ^ f);
            }
        }
        BCK(hipMemcpyAsync(b->d_pa[f], pa.data(), n * sizeof(KParams<T>), hipMemcpyHostToDevice, b->stream));
        BCK(hipMemcpyAsync(b->d_pb[f], pb.data(), n * sizeof(KParams<T>), hipMemcpyHostToDevice, b->stream));
    }
    // the staging vectors must live until the copies are done
    BCK(hipStreamSynchronize(b->stream));
    return MPX_OK;
}

template <typename T>
mpx_status batch_body(mpx_batch *b, int f) {
    const KParams<T> *pa = (const KParams<T> *)b->d_pa[f];
    const KParams<T> *pb = (const KParams<T> *)b->d_pb[f];
    hipStream_t st = b->stream;
    if (b->variant == 0) {
        // E pass, film half steps and probes, then the bulk H pass (which
        // moves every instance's step counter)
        BCK(launch_epass_batch<T>(pa, b->d_work2, b->nwork2, b->d_wmixed, b->nwmixed, b->any_xcls, st));
        BCK(launch_film_batch<T>(pa, b->d_wext, b->nwext, b->d_wfilm, b->nwfilm, 1, 0, st));
        BCK(launch_probes_batch<T>(pa, b->d_wprobe, b->nwprobe, b->probe_maxpart, st));
        BCK(launch_film_batch<T>(pa, b->d_wext, b->nwext, b->d_wfilm, b->nwfilm, 2, 0, st));
        BCK(launch_hbulk_batch<T>(pa, b->d_work2, b->nwork2, 2, 1, st));
        return MPX_OK;
    }
    if (b->variant == 1)
        BCK(launch_sweep_batch<T>(pa, b->d_work, b->nwork, st));
    else
        BCK(launch_fused_batch<T>(pa, b->d_work, b->nwork, b->variant - 1, st));
    BCK(launch_film_batch<T>(pb, b->d_wext, b->nwext, b->d_wfilm, b->nwfilm, 1, 0, st));
    BCK(launch_probes_batch<T>(pb, b->d_wprobe, b->nwprobe, b->probe_maxpart, st));
    BCK(launch_film_batch<T>(pb, b->d_wext, b->nwext, b->d_wfilm, b->nwfilm, 2, 1, st));
    BCK(launch_tick_batch<T>(pb, b->d_tick, b->ntick, st));
    return MPX_OK;
}

template <typename T>
mpx_status batch_steps(mpx_batch *b, long long nsteps) {
    hipStream_t st = b->stream;
    mpx_status r;
    if ((r = batch_params<T>(b)) != MPX_OK) return r;
    // bracket half step of every instance
    for (mpx_sim *s : b->sims) {
        KParams<T> p;
        fill_params<T>(s, p, MODE_INPLACE, s->parity);
        BCK(launch_film<T>(p, s->nblk, 1, 0, st));
        BCK(launch_commit<T>(p, s->nblk, st));
        BCK(launch_hbulk<T>(p, 1, 0, st));
    }
    long long body = nsteps - 1;
    int f = 0;
    const int G = (b->graph_steps + 1) / 2 * 2;
    if (G > 0 && body >= G) {
        if (!b->graph_valid) {
            BCK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            for (int n = 0; n < G; n++) {
                r = batch_body<T>(b, b->variant == 0 ? 0 : (n & 1));
                if (r != MPX_OK) {
                    hipGraph_t g;
                    (void)hipStreamEndCapture(st, &g);
                    return r;
                }
            }
            BCK(hipStreamEndCapture(st, &b->graph));
            BCK(hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
            b->graph_valid = true;
        }
        while (body >= G) {
            BCK(hipGraphLaunch(b->gexec, st));
            body -= G;
        }
    }
    for (long long n = 0; n < body; n++) {
        if ((r = batch_body<T>(b, f)) != MPX_OK) return r;
        if (b->variant != 0) f ^= 1;
    }
    // the flips of the fused body: every instance changed parity (nsteps - 1) times
    if (b->variant != 0)
        for (mpx_sim *s : b->sims) s->parity ^= (int)((nsteps - 1) & 1);
    for (mpx_sim *s : b->sims) {
        if ((r = run_last<T>(s, s->parity, st)) != MPX_OK) {
            b->dead = true;
            b->err = s->err;
            return r;
        }
        s->step += nsteps;
    }
    return MPX_OK;
}

} // namespace

// ===========================================================================
// Adjoint: reverse-mode gradients of a film-energy loss
// ===========================================================================
namespace {

size_t psi_count(const mpx_sim *s, int a) {
    const int S = s->nlo[a] + s->nhi[a];
    return a == 0 ? (size_t)S * s->n[1] * s->n[2]
                  : a == 1 ? (size_t)s->px * S * s->n[2] : (size_t)s->px * s->n[1] * S;
}

// a full state at an integer time (the current buffer set of a handle)
struct Snap {
    void *E[3] = {}, *H[3] = {}, *psiE[3][3] = {}, *psiH[3][3] = {};
    std::vector<double *> M;
    long long step = 0;
};

void snap_free(Snap &z) {
    for (int c = 0; c < 3; c++) {
        (void)hipFree(z.E[c]);
        (void)hipFree(z.H[c]);
        for (int a = 0; a < 3; a++) {
            (void)hipFree(z.psiE[c][a]);
            (void)hipFree(z.psiH[c][a]);
        }
    }
    for (double *m : z.M) (void)hipFree(m);
    z = Snap();
}

mpx_status snap_alloc(mpx_sim *s, Snap &z) {
    for (int c = 0; c < 3; c++) {
        CK(hipMalloc(&z.E[c], s->nslot * s->esz));
        CK(hipMalloc(&z.H[c], s->nslot * s->esz));
        for (int a = 0; a < 3; a++)
            if (s->psiE[c][a]) {
                CK(hipMalloc(&z.psiE[c][a], psi_count(s, a) * s->esz));
                CK(hipMalloc(&z.psiH[c][a], psi_count(s, a) * s->esz));
            }
    }
    for (auto &f : s->films) {
        double *m = nullptr;
        CK(hipMalloc(&m, 9 * f.ns * sizeof(double)));
        z.M.push_back(m);
    }
    return MPX_OK;
}

// save (handle -> snapshot) or load (snapshot -> handle); e_only: E and its
// psi only
mpx_status snap_copy(mpx_sim *s, Snap &z, bool save, bool e_only = false) {
    hipStream_t st = s->stream;
    const size_t fb = s->nslot * s->esz;
    auto cp = [&](void *handle, void *snap, size_t bytes) -> mpx_status {
        CK(hipMemcpyAsync(save ? snap : handle, save ? handle : snap, bytes, hipMemcpyDeviceToDevice, st));
        return MPX_OK;
    };
    mpx_status r;
    for (int c = 0; c < 3; c++) {
        if ((r = cp(Eset(s, s->parity)[c], z.E[c], fb)) != MPX_OK) return r;
        for (int a = 0; a < 3; a++)
            if (s->psiE[c][a])
                if ((r = cp(psiEset(s, s->parity, c, a), z.psiE[c][a], psi_count(s, a) * s->esz)) != MPX_OK) return r;
    }
    if (e_only) return MPX_OK;
    for (int c = 0; c < 3; c++) {
        if ((r = cp(Hset(s, s->parity)[c], z.H[c], fb)) != MPX_OK) return r;
        for (int a = 0; a < 3; a++)
            if (s->psiH[c][a])
                if ((r = cp(s->psiH[c][a], z.psiH[c][a], psi_count(s, a) * s->esz)) != MPX_OK) return r;
    }
    for (size_t f = 0; f < s->films.size(); f++)
        if ((r = cp(s->films[f].M, z.M[f], 9 * s->films[f].ns * sizeof(double))) != MPX_OK) return r;
    if (save) {
        z.step = s->step;
    } else {
        s->step = z.step;
        CK(launch_set_step(s->d_step, z.step, st));
    }
    return MPX_OK;
}

// adjoint arrays
struct AdjHost {
    void *lE[3] = {}, *lH[3] = {}, *lpsiE[3][3] = {}, *lpsiH[3][3] = {};
    void *aD[3][2] = {}, *eD[3][2] = {};
    double *gca[3] = {}, *gcb[3] = {};
    std::vector<AdjFilmDev> af;
    AdjFilmDev *d_af = nullptr;
    AdjFilmDev *d_af2 = nullptr; // tape schedule: lM and lMout swapped
    double *d_part = nullptr, *d_loss = nullptr, *d_out = nullptr;
    double *gbox_a = nullptr, *gbox_b = nullptr; // tape schedule: dL/dca, dL/dcb over the eps box's edges
    long long *d_seg0 = nullptr;                 // tape schedule: first step of the segment in hand
    void *lpsiH2[3][3] = {}, *lpsiE2[3][3] = {};  // tape schedule: second lambda psi sets
    uint8_t *d_aflags = nullptr;
    void *mu[3] = {};
    std::vector<double *> aDr, aDr2; // per film: the reach's curl-part table of each half step of a step
    std::vector<long long> film_nr;
};

void adj_free(AdjHost &h) {
    for (int c = 0; c < 3; c++) {
        (void)hipFree(h.lE[c]);
        (void)hipFree(h.lH[c]);
        (void)hipFree(h.gca[c]);
        (void)hipFree(h.gcb[c]);
        for (int a = 0; a < 3; a++) {
            (void)hipFree(h.lpsiE[c][a]);
            (void)hipFree(h.lpsiH[c][a]);
        }
        for (int w = 0; w < 2; w++) {
            (void)hipFree(h.aD[c][w]);
            (void)hipFree(h.eD[c][w]);
        }
    }
    for (auto &g : h.af) {
        (void)hipFree(g.lM);
        (void)hipFree(g.lMout);
        (void)hipFree(g.lp);
        (void)hipFree(g.lq);
        (void)hipFree(g.gMs);
        (void)hipFree(g.gH0);
    }
    (void)hipFree(h.d_af);
    (void)hipFree(h.d_af2);
    for (int c = 0; c < 3; c++)
        for (int a = 0; a < 3; a++) {
            (void)hipFree(h.lpsiH2[c][a]);
            (void)hipFree(h.lpsiE2[c][a]);
        }
    (void)hipFree(h.d_aflags);
    for (int c = 0; c < 3; c++) (void)hipFree(h.mu[c]);
    for (double *d : h.aDr) (void)hipFree(d);
    for (double *d : h.aDr2) (void)hipFree(d);
    (void)hipFree(h.gbox_a);
    (void)hipFree(h.gbox_b);
    (void)hipFree(h.d_seg0);
    (void)hipFree(h.d_part);
    (void)hipFree(h.d_loss);
    (void)hipFree(h.d_out);
    h = AdjHost();
}

// full_eps: the plain schedule's per-edge dL/dca, dL/dcb and curl-part
// adjoint arrays (the tape schedule keeps box accumulators and computes the
// curl parts on the fly)
mpx_status adj_alloc(mpx_sim *s, AdjHost &h, long long nout, bool full_eps = true) {
    const size_t fb = s->nslot * s->esz;
    auto z = [&](void **p, size_t bytes) -> mpx_status {
        CK(hipMalloc(p, std::max<size_t>(bytes, 8)));
        CK(hipMemsetAsync(*p, 0, std::max<size_t>(bytes, 8), s->stream));
        return MPX_OK;
    };
    mpx_status r;
    for (int c = 0; c < 3; c++) {
        if ((r = z(&h.lE[c], fb)) != MPX_OK || (r = z(&h.lH[c], fb)) != MPX_OK) return r;
        if (full_eps) {
            if ((r = z((void **)&h.gca[c], s->nslot * sizeof(double))) != MPX_OK) return r;
            if ((r = z((void **)&h.gcb[c], s->nslot * sizeof(double))) != MPX_OK) return r;
        }
        if (full_eps)
            for (int w = 0; w < 2; w++)
                if ((r = z(&h.aD[c][w], fb)) != MPX_OK || (r = z(&h.eD[c][w], fb)) != MPX_OK) return r;
        for (int a = 0; a < 3; a++)
            if (s->psiE[c][a]) {
                if ((r = z(&h.lpsiE[c][a], psi_count(s, a) * s->esz)) != MPX_OK) return r;
                if ((r = z(&h.lpsiH[c][a], psi_count(s, a) * s->esz)) != MPX_OK) return r;
            }
    }
    for (auto &f : s->films) {
        AdjFilmDev g{};
        if ((r = z((void **)&g.lM, 9 * f.ns * sizeof(double))) != MPX_OK) return r;
        if ((r = z((void **)&g.lMout, 9 * f.ns * sizeof(double))) != MPX_OK) return r;
        if ((r = z((void **)&g.lp, 9 * f.ns * sizeof(double))) != MPX_OK) return r;
        if ((r = z((void **)&g.lq, 9 * f.ns * sizeof(double))) != MPX_OK) return r;
        if ((r = z((void **)&g.gMs, 3 * f.ns * sizeof(double))) != MPX_OK) return r;
        if ((r = z((void **)&g.gH0, 9 * f.ns * sizeof(double))) != MPX_OK) return r;
        h.af.push_back(g);
    }
    if (!h.af.empty()) {
        CK(hipMalloc(&h.d_af, h.af.size() * sizeof(AdjFilmDev)));
        CK(hipMemcpy(h.d_af, h.af.data(), h.af.size() * sizeof(AdjFilmDev), hipMemcpyHostToDevice));
    }
    const long long nb = (long long)((s->n[0] + 63) / 64) * ((s->n[1] + 3) / 4) * s->n[2];
    if ((r = z((void **)&h.d_part, nb * sizeof(double))) != MPX_OK) return r;
    if ((r = z((void **)&h.d_loss, sizeof(double))) != MPX_OK) return r;
    if ((r = z((void **)&h.d_out, std::max<long long>(1, nout) * sizeof(double))) != MPX_OK) return r;
    return MPX_OK;
}

template <typename T>
void adj_params(const mpx_sim *s, const AdjHost &h, AdjParams<T> &A) {
    fill_params<T>(s, A.p, MODE_INPLACE, s->parity);
    for (int c = 0; c < 3; c++) {
        A.lE[c] = (T *)h.lE[c];
        A.lH[c] = (T *)h.lH[c];
        A.gca[c] = h.gca[c];
        A.gcb[c] = h.gcb[c];
        for (int a = 0; a < 3; a++) {
            A.lpsiE[c][a] = (T *)h.lpsiE[c][a];
            A.lpsiH[c][a] = (T *)h.lpsiH[c][a];
        }
        for (int w = 0; w < 2; w++) {
            A.aD[c][w] = (T *)h.aD[c][w];
            A.eD[c][w] = (T *)h.eD[c][w];
        }
    }
    A.af = h.d_af;
}

// the bracket half step of the step driver (first H/M half step, in place)
template <typename T>
mpx_status half_step_inplace(mpx_sim *s) {
    KParams<T> p;
    fill_params<T>(s, p, MODE_INPLACE, s->parity);
    CK(launch_film<T>(p, s->nblk, 1, 0, s->stream));
    CK(launch_commit<T>(p, s->nblk, s->stream));
    CK(launch_hbulk<T>(p, 1, 0, s->stream));
    return MPX_OK;
}

// dL/dH0 and dL/dMs per cell of ms_box from the films' per-face sums (seed
// scale S divided out)
mpx_status film_grads(mpx_sim *s, const AdjHost &h, double S, const int *ms_box, double *gH0, double *gms) {
    gH0[0] = gH0[1] = gH0[2] = 0.0;
    std::vector<std::vector<double>> gf(s->films.size());
    for (size_t f = 0; f < s->films.size(); f++) {
        const FilmHost &F = s->films[f];
        std::vector<double> v(9 * F.ns);
        CK(hipMemcpy(v.data(), h.af[f].gH0, v.size() * sizeof(double), hipMemcpyDeviceToHost));
        for (int c = 0; c < 3; c++)
            for (int w = 0; w < 3; w++)
                for (long long l = 0; l < F.ns; l++) gH0[w] += v[(c * 3 + w) * F.ns + l] / S;
        gf[f].resize(3 * F.ns);
        CK(hipMemcpy(gf[f].data(), h.af[f].gMs, gf[f].size() * sizeof(double), hipMemcpyDeviceToHost));
    }
    const long long nms = (long long)ms_box[3] * ms_box[4] * ms_box[5];
    for (long long t = 0; t < nms; t++) {
        const int cc[3] = {ms_box[0] + (int)(t % ms_box[3]), ms_box[1] + (int)((t / ms_box[3]) % ms_box[4]),
                           ms_box[2] + (int)(t / ((long long)ms_box[3] * ms_box[4]))};
        double g = 0.0;
        // the cell's two faces of each family: Ms of a face is the mean over
        // its in-domain cells
        for (int c = 0; c < 3; c++)
            for (int u = 0; u < 2; u++) {
                int fi[3] = {cc[0], cc[1], cc[2]};
                fi[c] += u;
                if (fi[c] >= s->n[c]) {
                    if (!s->per[c]) continue;
                    fi[c] -= s->n[c];
                }
                for (size_t f = 0; f < s->films.size(); f++) {
                    const FilmHost &F = s->films[f];
                    const int r0 = fi[0] - F.b0[0], r1 = fi[1] - F.b0[1], r2 = fi[2] - F.b0[2];
                    if (r0 < 0 || r0 >= F.bn[0] || r1 < 0 || r1 >= F.bn[1] || r2 < 0 || r2 >= F.bn[2]) continue;
                    const long long l = r0 + (long long)F.bn[0] * (r1 + (long long)F.bn[1] * r2);
                    int cnt = 0;
                    for (int uu = -1; uu <= 0; uu++) {
                        int q3[3] = {fi[0], fi[1], fi[2]};
                        q3[c] += uu;
                        if (cell_id_h(s, q3[0], q3[1], q3[2]) >= 0) cnt++;
                    }
                    if (cnt) g += gf[f][c * F.ns + l] / cnt;
                    break;
                }
            }
        gms[t] = g / S;
    }
    return MPX_OK;
}

// whether two cell boxes (x0, y0, z0, nx, ny, nz) share a cell
bool boxes_meet(const int *a, const int *b) {
    for (int i = 0; i < 3; i++)
        if (a[i] + a[3 + i] <= b[i] || b[i] + b[3 + i] <= a[i]) return false;
    return a[3] * a[4] * a[5] > 0 && b[3] * b[4] * b[5] > 0;
}

// adds the film-energy loss's own eps_r term (accumulated per cell of the
// film's cell box cb, scaled like the adjoint seed) to the eps-box gradient
mpx_status add_loss_eps(mpx_sim *s, const double *d_acc, const int *cb, const int *eps_box, double *geps) {
    const long long nc = (long long)cb[3] * cb[4] * cb[5];
    std::vector<double> acc(nc);
    CK(hipMemcpy(acc.data(), d_acc, nc * sizeof(double), hipMemcpyDeviceToHost));
    const long long neps = (long long)eps_box[3] * eps_box[4] * eps_box[5];
    for (long long t = 0; t < neps; t++) {
        const int c[3] = {eps_box[0] + (int)(t % eps_box[3]), eps_box[1] + (int)((t / eps_box[3]) % eps_box[4]),
                          eps_box[2] + (int)(t / ((long long)eps_box[3] * eps_box[4]))};
        int l[3];
        bool in = true;
        for (int a = 0; a < 3; a++) {
            l[a] = c[a] - cb[a];
            if (l[a] < 0 || l[a] >= cb[3 + a]) in = false;
        }
        if (in) geps[t] += acc[l[0] + (long long)cb[3] * (l[1] + (long long)cb[4] * l[2])];
    }
    return MPX_OK;
}

template <typename T>
mpx_status run_adjoint(mpx_sim *s, long long N, long long loss_from, int film, int K, const int *eps_box,
                       const int *ms_box, double *loss, double *gH0, double *geps, double *gms) {
    hipStream_t st = s->stream;
    const int saved_fused = s->fused;
    s->fused = 0; // one step at a time, in place
    const long long step0 = s->step;
    const int ncp = (int)((N + K - 1) / K);
    std::vector<Snap> cp(ncp), seg(K);
    Snap fin;
    AdjHost h;
    const long long neps = (long long)eps_box[3] * eps_box[4] * eps_box[5];
    mpx_status r = MPX_OK;
    double *d_lacc = nullptr; // the loss's own eps_r term per film cell
    const int *fcb = s->films[film].cb;
    auto body = [&]() -> mpx_status {
        mpx_status q;
        if ((q = adj_alloc(s, h, neps)) != MPX_OK) return q;
        if (boxes_meet(eps_box, fcb)) {
            const size_t nb = (size_t)fcb[3] * fcb[4] * fcb[5] * sizeof(double);
            CK(hipMalloc(&d_lacc, nb));
            CK(hipMemsetAsync(d_lacc, 0, nb, st));
        }
        for (auto &z : cp)
            if ((q = snap_alloc(s, z)) != MPX_OK) return q;
        for (int m = 1; m < K; m++)
            if ((q = snap_alloc(s, seg[m])) != MPX_OK) return q;
        if ((q = snap_alloc(s, fin)) != MPX_OK) return q;
        const double dt = s->dt;
        // forward with checkpoints and the loss
        for (long long n = 0; n < N; n++) {
            if (n % K == 0 && (q = snap_copy(s, cp[n / K], true)) != MPX_OK) return q;
            if ((q = enqueue_steps<T>(s, 1)) != MPX_OK) return q;
            s->step += 1;
            if (n + 1 > loss_from) {
                KParams<T> p;
                fill_params<T>(s, p, MODE_INPLACE, s->parity);
                CK(launch_film_energy<T>(p, film, h.d_part, h.d_loss, dt, st));
            }
        }
        if ((q = snap_copy(s, fin, true)) != MPX_OK) return q;
        CK(hipMemcpyAsync(loss, h.d_loss, sizeof(double), hipMemcpyDeviceToHost, st));
        CK(hipStreamSynchronize(st));
        // The adjoint is linear in its seed: seed it with S dL/d(state), S a
        // power of two near 1/L, so that the adjoint fields sit near unit
        // scale instead of at the loss's SI magnitude (a float32 run would
        // otherwise underflow), and divide the gradients by S at the end.
        // In float64 the scaling is exact.
        double S = 1.0;
        if (std::isfinite(*loss) && *loss > 0.0) S = std::ldexp(1.0, -std::ilogb(*loss));
        // reverse, segment by segment
        for (int g = ncp - 1; g >= 0; g--) {
            const long long c0 = (long long)g * K, c1 = std::min<long long>(c0 + K, N);
            if ((q = snap_copy(s, cp[g], false)) != MPX_OK) return q;
            for (long long m = 1; m < c1 - c0; m++) {
                if ((q = enqueue_steps<T>(s, 1)) != MPX_OK) return q;
                s->step += 1;
                if ((q = snap_copy(s, seg[m], true)) != MPX_OK) return q;
            }
            for (long long n = c1 - 1; n >= c0; n--) {
                Snap &Sn = n == c0 ? cp[g] : seg[n - c0];
                Snap &Sp = n + 1 < c1 ? seg[n + 1 - c0] : (g + 1 < ncp ? cp[g + 1] : fin);
                AdjParams<T> A;
                if (n + 1 > loss_from) {
                    if ((q = snap_copy(s, Sp, false)) != MPX_OK) return q;
                    adj_params<T>(s, h, A);
                    CK(launch_adj_loss<T>(A, film, dt * S, st));
                    if (d_lacc) {
                        KParams<T> p;
                        fill_params<T>(s, p, MODE_INPLACE, s->parity);
                        CK(launch_adj_loss_eps_state<T>(p, film, dt * S, d_lacc, st, fcb));
                    }
                }
                // the step's intermediate states
                if ((q = snap_copy(s, Sn, false)) != MPX_OK) return q;
                if ((q = half_step_inplace<T>(s)) != MPX_OK) return q;
                {
                    KParams<T> p;
                    fill_params<T>(s, p, MODE_INPLACE, s->parity);
                    CK(launch_epass<T>(p, st));
                }
                // second half step: input (E^{n+1}, H^{n+1/2}, M^{n+1/2})
                adj_params<T>(s, h, A);
                CK(launch_bhat<T>(A.p, 1, st));
                CK(launch_adj_half<T>(A, s->nblk, st));
                // E step: input H^{n+1/2}, E^n and its psi
                if ((q = snap_copy(s, Sn, false, true)) != MPX_OK) return q;
                adj_params<T>(s, h, A);
                CK(launch_adj_estep<T>(A, st));
                // first half step: input S_n
                if ((q = snap_copy(s, Sn, false)) != MPX_OK) return q;
                adj_params<T>(s, h, A);
                CK(launch_bhat<T>(A.p, 1, st));
                CK(launch_adj_half<T>(A, s->nblk, st));
            }
        }
        // the initial magnetisation M0 = Ms u
        if (step0 == 0 && s->have_u)
            CK(launch_adj_init_ms(s->d_blocktab, s->nblk, s->d_films, h.d_af, s->u, st));
        // dL/d eps_r over the box
        {
            AdjParams<T> A;
            adj_params<T>(s, h, A);
            CK(launch_adj_eps<T>(A, eps_box, h.d_out, st));
            if (neps > 0) CK(hipMemcpyAsync(geps, h.d_out, neps * sizeof(double), hipMemcpyDeviceToHost, st));
        }
        CK(hipStreamSynchronize(st));
        if (d_lacc && (q = add_loss_eps(s, d_lacc, fcb, eps_box, geps)) != MPX_OK) return q;
        for (long long t = 0; t < neps; t++) geps[t] /= S;
        if ((q = film_grads(s, h, S, ms_box, gH0, gms)) != MPX_OK) return q;
        // leave the handle at the end of the forward run
        if ((q = snap_copy(s, fin, false)) != MPX_OK) return q;
        CK(hipStreamSynchronize(st));
        return MPX_OK;
    };
    r = body();
    s->fused = saved_fused;
    if (d_lacc) {
        (void)hipStreamSynchronize(st);
        (void)hipFree(d_lacc);
    }
    adj_free(h);
    for (auto &z : cp) snap_free(z);
    for (auto &z : seg) snap_free(z);
    snap_free(fin);
    return r;
}

// ---------------------------------------------------------------------------
// tape schedule
//
// Forward: the plain stepping path (merged pairs, graphs) with a temporary
// film-energy probe for the loss and a full snapshot every K steps.
// Reverse, segment by segment: reload the segment's snapshot, recompute its
// steps once with the merged-pair kernels while writing a tape of what the
// adjoint maps read (the film's M and prepass values of both half steps, the
// film region's E and H at each integer time, E^n and the curl input x^n over
// the eps box), then run the adjoint maps of the segment's steps backwards
// from the tape: no forward work and no full-state copy inside the reverse
// sweep.  Every full segment launches the same kernels with the same
// arguments (the tape is reused; the step index lives on the device), so one
// captured graph serves them all.
// ---------------------------------------------------------------------------

// a full state at an integer time in one allocation, and its copy tables
struct Snap2 {
    char *buf = nullptr;
    long long step = 0;
};

struct SnapLayout {
    std::vector<void *> handle; // handle-side arrays, in layout order
    std::vector<size_t> off, bytes;
    std::vector<int> film_of;   // film index of an M segment, -1 otherwise
    size_t total = 0;
    int nblk = 1;
};

SnapLayout snap_layout(const mpx_sim *s) {
    SnapLayout L;
    auto add = [&](void *h, size_t b, int f) {
        L.handle.push_back(h);
        L.off.push_back(L.total);
        L.bytes.push_back(b);
        L.film_of.push_back(f);
        L.total += (b + 255) / 256 * 256;
        L.nblk = std::max<int>(L.nblk, (int)std::min<size_t>(2048, (b / 16 + 255) / 256));
    };
    const size_t fb = s->nslot * s->esz;
    for (int c = 0; c < 3; c++) add(Eset(s, s->parity)[c], fb, -1);
    for (int c = 0; c < 3; c++) add(Hset(s, s->parity)[c], fb, -1);
    for (int c = 0; c < 3; c++)
        for (int a = 0; a < 3; a++)
            if (s->psiE[c][a]) {
                add(psiEset(s, s->parity, c, a), psi_count(s, a) * s->esz, -1);
                add(s->psiH[c][a], psi_count(s, a) * s->esz, -1);
            }
    for (size_t f = 0; f < s->films.size(); f++) add(s->films[f].M, 9 * s->films[f].ns * sizeof(double), (int)f);
    return L;
}

struct Tape {
    int K = 0, nf = 0;
    char *buf = nullptr;
    size_t bytes = 0;
    std::vector<double *> Mf, Mh, B1s, B1n, B2s, B2n; // [f][slot]
    double *loss = nullptr, *box = nullptr;
    long long loss_sz = 0, box_sz = 0;
    FilmDev *d_var = nullptr;
    CopySeg *d_tab = nullptr; // copy tables: per snapshot save, load, load-to-tape
    int nseg = 0;
    double *lossp(int m) const { return loss + (size_t)m * loss_sz; }
    double *boxp(int m) const { return box + (size_t)m * box_sz; }
};
enum { V_P1 = 0, V_P2, V_C, V_R1, V_BR, V_BRC, NV };

void tape_free(Tape &t) {
    (void)hipFree(t.buf);
    (void)hipFree(t.d_var);
    (void)hipFree(t.d_tab);
    t = Tape();
}

mpx_status tape_alloc(mpx_sim *s, Tape &t, int K, const int *film_cb, const int *eps_box) {
    t.K = K;
    t.nf = (int)s->films.size();
    const int nf = t.nf;
    t.loss_sz = film_tape_size(film_cb);
    t.box_sz = (long long)eps_box[3] * eps_box[4] * eps_box[5] > 0 ? box_tape_size(eps_box) : 0;
    // layout: per film the M slots (K + 1 integer-time, K half-time) and the
    // prepass slots, then the loss and box tapes
    size_t off = 0;
    std::vector<size_t> o;
    auto put = [&](size_t bytes) {
        o.push_back(off);
        off += (bytes + 255) / 256 * 256;
    };
    for (int f = 0; f < nf; f++) {
        const FilmHost &F = s->films[f];
        for (int m = 0; m <= K; m++) put(9 * F.ns * sizeof(double));
        for (int m = 0; m < K; m++) put(9 * F.ns * sizeof(double));
        for (int m = 0; m < K; m++)
            for (int w = 0; w < 4; w++) put(3 * F.nse * sizeof(double));
    }
    put((size_t)K * t.loss_sz * sizeof(double));
    put((size_t)std::max<long long>(1, K * t.box_sz) * sizeof(double));
    CK(hipMalloc(&t.buf, off));
    CK(hipMemsetAsync(t.buf, 0, off, s->stream));
    t.bytes = off;
    size_t q = 0;
    t.Mf.assign((size_t)nf * (K + 1), nullptr);
    t.Mh.assign((size_t)nf * K, nullptr);
    t.B1s = t.B1n = t.B2s = t.B2n = std::vector<double *>((size_t)nf * K, nullptr);
    for (int f = 0; f < nf; f++) {
        for (int m = 0; m <= K; m++) t.Mf[(size_t)f * (K + 1) + m] = (double *)(t.buf + o[q++]);
        for (int m = 0; m < K; m++) t.Mh[(size_t)f * K + m] = (double *)(t.buf + o[q++]);
        for (int m = 0; m < K; m++) {
            t.B1s[(size_t)f * K + m] = (double *)(t.buf + o[q++]);
            t.B1n[(size_t)f * K + m] = (double *)(t.buf + o[q++]);
            t.B2s[(size_t)f * K + m] = (double *)(t.buf + o[q++]);
            t.B2n[(size_t)f * K + m] = (double *)(t.buf + o[q++]);
        }
    }
    t.loss = (double *)(t.buf + o[q++]);
    t.box = (double *)(t.buf + o[q++]);
    // film descriptors per slot and use
    std::vector<FilmDev> base(nf), var((size_t)K * NV * nf);
    if (nf) CK(hipMemcpy(base.data(), s->d_films, nf * sizeof(FilmDev), hipMemcpyDeviceToHost));
    for (int m = 0; m < K; m++)
        for (int f = 0; f < nf; f++) {
            auto Mf = [&](int mm) { return t.Mf[(size_t)f * (K + 1) + mm]; };
            auto Mh = [&](int mm) { return t.Mh[(size_t)f * K + std::min(mm, K - 1)]; };
            auto B1s = [&](int mm) { return t.B1s[(size_t)f * K + std::min(mm, K - 1)]; };
            auto B1n = [&](int mm) { return t.B1n[(size_t)f * K + std::min(mm, K - 1)]; };
            const size_t i0 = (size_t)m * NV * nf + f;
            FilmDev d;
            // HALF2 of step m: reads M^{n+1/2}, writes M^{n+1}, its prepass and
            // (unless it ends the segment) the prepass of HALF1 of step m + 1
            d = base[f];
            d.M = Mh(m);
            d.M1 = Mf(m + 1);
            d.Bs = t.B2s[(size_t)f * K + m];
            d.Bn = t.B2n[(size_t)f * K + m];
            d.Bs2 = m + 1 < K ? B1s(m + 1) : nullptr;
            d.Bn2 = m + 1 < K ? B1n(m + 1) : nullptr;
            var[i0 + V_P1 * nf] = d;
            // HALF1 of step m + 1 (merged pair): reads M^{n+1} and its prepass,
            // writes M^{n+3/2}
            d = base[f];
            d.M = Mh(m + 1);
            d.M1 = Mf(m + 1);
            d.Bs = d.Bs2 = B1s(m + 1);
            d.Bn = d.Bn2 = B1n(m + 1);
            var[i0 + V_P2 * nf] = d;
            // commit after the segment's last HALF2 (copies M^{n+1} onto itself)
            d = base[f];
            d.M = d.M1 = Mf(m + 1);
            var[i0 + V_C * nf] = d;
            // the adjoint of HALF1 of step m: M^n and its prepass
            d = base[f];
            d.M = Mf(m);
            d.Bs = B1s(m);
            d.Bn = B1n(m);
            d.Bs2 = d.Bn2 = nullptr;
            var[i0 + V_R1 * nf] = d;
            // the bracket (HALF1 of the segment's first step) and its commit
            d = base[f];
            d.M = Mf(0);
            d.M1 = Mh(0);
            d.Bs = B1s(0);
            d.Bn = B1n(0);
            d.Bs2 = d.Bn2 = nullptr;
            var[i0 + V_BR * nf] = d;
            d = base[f];
            d.M = d.M1 = Mh(0);
            var[i0 + V_BRC * nf] = d;
        }
    if (nf) {
        CK(hipMalloc(&t.d_var, var.size() * sizeof(FilmDev)));
        CK(hipMemcpy(t.d_var, var.data(), var.size() * sizeof(FilmDev), hipMemcpyHostToDevice));
    }
    return MPX_OK;
}

const FilmDev *tvar(const Tape &t, int m, int v) { return t.d_var ? t.d_var + ((size_t)m * NV + v) * t.nf : nullptr; }

// copy tables of every snapshot: [snapshot][save | load | load-to-tape][segment]
mpx_status snap_tables(mpx_sim *s, Tape &t, const SnapLayout &L, const std::vector<Snap2 *> &snaps) {
    const int ns = (int)L.handle.size();
    t.nseg = ns;
    std::vector<CopySeg> tab((size_t)snaps.size() * 3 * ns);
    for (size_t z = 0; z < snaps.size(); z++)
        for (int q = 0; q < ns; q++) {
            char *sp = snaps[z]->buf + L.off[q];
            void *h = L.handle[q];
            const long long b = (long long)L.bytes[q];
            tab[(z * 3 + 0) * ns + q] = CopySeg{h, sp, b};
            tab[(z * 3 + 1) * ns + q] = CopySeg{sp, h, b};
            void *ht = L.film_of[q] >= 0 ? (void *)t.Mf[(size_t)L.film_of[q] * (t.K + 1)] : h;
            tab[(z * 3 + 2) * ns + q] = CopySeg{sp, ht, b};
        }
    CK(hipMalloc(&t.d_tab, std::max<size_t>(1, tab.size()) * sizeof(CopySeg)));
    CK(hipMemcpy(t.d_tab, tab.data(), tab.size() * sizeof(CopySeg), hipMemcpyHostToDevice));
    return MPX_OK;
}

// the loss of an adjoint run: kind 0, dt times the film-energy sum over the
// steps after loss_from; kind 1, a weighted sum of one E component's values at
// one edge, L = sum_i w[i] E(t_{i+1}) (host weights, one per step)
struct AdjLoss {
    int kind = 0;
    int film = 0;
    long long loss_from = 0;
    int field = 0, ijk[3] = {0, 0, 0};
    const double *w = nullptr;
};

template <typename T>
mpx_status run_adjoint_tape(mpx_sim *s, long long N, const AdjLoss &ls, int K, const int *eps_box, const int *ms_box,
                            double *loss, double *gH0, double *geps, double *gms) {
    hipStream_t st = s->stream;
    const int saved_fused = s->fused;
    s->fused = 0;
    const long long step0 = s->step;
    const int ncp = (int)((N + K - 1) / K);
    const long long neps = (long long)eps_box[3] * eps_box[4] * eps_box[5];
    const int nblk = s->nblk;
    const int film = ls.film;
    const long long loss_from = ls.loss_from;
    const bool floss = ls.kind == 0; // the film-energy loss (its tapes and terms)
    static const FilmHost no_film{};
    const FilmHost &LF = floss ? s->films[film] : no_film;
    double *d_w = nullptr;
    std::vector<Snap2> cp(ncp);
    Snap2 fin;
    AdjHost h;
    Tape tp;
    // captured segments: 0 the forward run with the tape and the probes, 1 a
    // recompute with the tape, 2 and 3 the reverse steps from lambda psiH set
    // 0 and set 1
    hipGraph_t graph[4] = {};
    hipGraphExec_t gexec[4] = {};
    char *pages = nullptr; // the tapes kept from the forward run
    bool probe_added = false;
    double *d_lacc = nullptr; // the film-energy loss's own eps_r term per film cell
    bool merge = s->adj_schedule == 0; // one field pass for the two half-step transposes around an integer time
    auto body = [&]() -> mpx_status {
        mpx_status q;
        if ((q = adj_alloc(s, h, neps, false)) != MPX_OK) return q;
        if (floss && boxes_meet(eps_box, LF.cb)) {
            const size_t nb = (size_t)LF.cb[3] * LF.cb[4] * LF.cb[5] * sizeof(double);
            CK(hipMalloc(&d_lacc, nb));
            CK(hipMemsetAsync(d_lacc, 0, nb, st));
        }
        for (int c = 0; c < 3; c++) {
            CK(hipMalloc(&h.mu[c], s->nslot * s->esz));
            CK(hipMemsetAsync(h.mu[c], 0, s->nslot * s->esz, st));
        }
        // second lambda psi sets (the field passes read one and write the other)
        for (int c = 0; c < 3; c++)
            for (int a = 0; a < 3; a++)
                if (s->psiE[c][a]) {
                    const size_t b = psi_count(s, a) * s->esz;
                    CK(hipMalloc(&h.lpsiH2[c][a], b));
                    CK(hipMalloc(&h.lpsiE2[c][a], b));
                    CK(hipMemsetAsync(h.lpsiH2[c][a], 0, b, st));
                    CK(hipMemsetAsync(h.lpsiE2[c][a], 0, b, st));
                }
        // each film's reach: its face box grown by one slot (a whole periodic
        // axis), with the table of its faces' curl-part adjoints
        for (size_t f = 0; f < h.af.size(); f++) {
            const FilmHost &F = s->films[f];
            AdjFilmDev &g = h.af[f];
            long long nr = 1;
            for (int a = 0; a < 3; a++) {
                if (s->per[a]) {
                    g.r0[a] = 0;
                    g.rn[a] = s->n[a];
                } else {
                    const int lo = std::max(0, F.b0[a] - 1), hi = std::min(s->n[a] - 1, F.b0[a] + F.bn[a]);
                    g.r0[a] = lo;
                    g.rn[a] = hi - lo + 1;
                }
                nr *= g.rn[a];
            }
            g.nr = nr;
            double *d = nullptr, *d2 = nullptr;
            CK(hipMalloc(&d, 6 * nr * sizeof(double)));
            CK(hipMalloc(&d2, 6 * nr * sizeof(double)));
            h.aDr.push_back(d);
            h.aDr2.push_back(d2);
            g.aDr = d;
            h.film_nr.push_back(nr);
        }
        // per-tile flags of the field passes: 1 CPML, 4 a film's reach, each
        // within two slots of the tile
        {
            const int nxt = (s->n[0] + kPassTX - 1) / kPassTX, nyt = (s->n[1] + kPassTY - 1) / kPassTY;
            const int nt = pass_tiles(s->n);
            std::vector<uint8_t> fl(nt, 0);
            for (int t = 0; t < nt; t++) {
                const int i0 = (t % nxt) * kPassTX, j0 = ((t / nxt) % nyt) * kPassTY, k = t / (nxt * nyt);
                const int lo[3] = {i0 - 2, j0 - 2, k - 2}, hi[3] = {i0 + kPassTX + 1, j0 + kPassTY + 1, k + 2};
                uint8_t fv = 0;
                for (int a = 0; a < 3; a++) {
                    if (s->nlo[a] > 0 && lo[a] < s->nlo[a]) fv |= 1;
                    if (s->nhi[a] > 0 && hi[a] >= s->n[a] - s->nhi[a]) fv |= 1;
                }
                for (auto &g : h.af) {
                    bool in = true;
                    for (int a = 0; a < 3; a++)
                        if (g.r0[a] + g.rn[a] <= lo[a] || g.r0[a] > hi[a]) in = false;
                    if (in) fv |= 4;
                }
                fl[t] = fv;
            }
            CK(hipMalloc(&h.d_aflags, ((size_t)nt + 4) / 4 * 4)); // whole words (read through the scalar cache)
            CK(hipMemcpy(h.d_aflags, fl.data(), nt, hipMemcpyHostToDevice));
        }
        // the merged reverse pass needs the films' reaches off the CPML slabs
        // (their faces keep no CPML state between half steps)
        for (auto &g : h.af)
            for (int a = 0; a < 3; a++) {
                if (s->nlo[a] > 0 && g.r0[a] < s->nlo[a]) merge = false;
                if (s->nhi[a] > 0 && g.r0[a] + g.rn[a] > s->n[a] - s->nhi[a]) merge = false;
            }
        if (!h.af.empty()) {
            CK(hipMemcpy(h.d_af, h.af.data(), h.af.size() * sizeof(AdjFilmDev), hipMemcpyHostToDevice));
            // lambda M ping-pong: the first map of a step reads lM and writes
            // lMout, the second reads lMout and writes lM
            std::vector<AdjFilmDev> af2 = h.af;
            for (size_t f = 0; f < af2.size(); f++) {
                std::swap(af2[f].lM, af2[f].lMout);
                af2[f].aDr = h.aDr2[f]; // the first half step's table (kept for the merged pass)
            }
            CK(hipMalloc(&h.d_af2, af2.size() * sizeof(AdjFilmDev)));
            CK(hipMemcpy(h.d_af2, af2.data(), af2.size() * sizeof(AdjFilmDev), hipMemcpyHostToDevice));
        }
        if (neps > 0) {
            const size_t gb = (size_t)box_tape_size(eps_box) / 2 * sizeof(double); // 3 components
            CK(hipMalloc(&h.gbox_a, gb));
            CK(hipMalloc(&h.gbox_b, gb));
            CK(hipMemsetAsync(h.gbox_a, 0, gb, st));
            CK(hipMemsetAsync(h.gbox_b, 0, gb, st));
        }
        CK(hipMalloc(&h.d_seg0, sizeof(long long)));
        if ((q = tape_alloc(s, tp, K, LF.cb, eps_box)) != MPX_OK) return q;
        const SnapLayout L = snap_layout(s);
        // the last npage segments keep the tape their forward run writes (a
        // page each: no checkpoint and no recompute); the others take a
        // checkpoint and are recomputed in the reverse sweep
        int npage = 0;
        if (s->adj_resident != 0) {
            const double page = (double)tp.bytes, snap = (double)L.total;
            if (s->adj_resident > 0) {
                npage = (int)std::min<double>(ncp, std::floor((double)s->adj_resident / page));
            } else {
                size_t fr = 0, tot = 0;
                CK(hipMemGetInfo(&fr, &tot));
                const double cap = 0.75 * (double)fr - snap; // less the final state's copy
                npage = ncp;
                while (npage > 0 && npage * page + (ncp - npage) * snap > cap) npage--;
            }
        }
        const int g0 = ncp - npage;
        std::vector<Snap2 *> all; // the checkpoints of segments 0 .. g0 - 1, then the final state
        for (int g = 0; g < g0; g++) {
            CK(hipMalloc(&cp[g].buf, L.total));
            all.push_back(&cp[g]);
        }
        CK(hipMalloc(&fin.buf, L.total));
        all.push_back(&fin);
        if (npage) CK(hipMalloc(&pages, (size_t)npage * tp.bytes));
        if ((q = snap_tables(s, tp, L, all)) != MPX_OK) return q;
        const int ns = tp.nseg;
        auto tab = [&](int z, int kind) { return tp.d_tab + ((size_t)z * 3 + kind) * ns; };
        const double dt = s->dt;
        const int nf = (int)s->films.size();
        auto mslot = [&](int f, int m) { return (void *)tp.Mf[(size_t)f * (K + 1) + m]; };
        auto mbytes = [&](int f) { return 9 * (size_t)s->films[f].ns * sizeof(double); };

        // a segment of len steps from an integer time with the tape (the
        // magnetisation in the tape's slots), with the probes in the forward
        // run; and the adjoint steps of a segment from its tape
        auto fwd = [&](int len, bool probes) -> mpx_status {
            KParams<T> p;
            fill_params<T>(s, p, MODE_INPLACE, s->parity);
            const int np = (int)s->probes.size();
            p.films = tvar(tp, 0, V_R1);
            if (floss) CK(launch_tape_loss<T>(p, film, 0, tp.lossp(0), st, LF.cb));
            p.films = tvar(tp, 0, V_BR);
            CK(launch_film<T>(p, nblk, 1, 0, st));
            p.films = tvar(tp, 0, V_BRC);
            CK(launch_commit<T>(p, nblk, st));
            CK(launch_hbulk<T>(p, 1, 0, st));
            for (int m = 0; m < len; m++) {
                if (neps > 0) CK(launch_tape_box<T>(p, eps_box, tp.boxp(m), st));
                CK(launch_epass<T>(p, st));
                p.films = tvar(tp, m, V_P1);
                CK(launch_film<T>(p, nblk, 1, 0, st));
                if (probes) CK(launch_probes<T>(p, np, s->probe_maxpart, st));
                if (m + 1 < len) {
                    if (floss) CK(launch_tape_loss<T>(p, film, 1, tp.lossp(m + 1), st, LF.cb));
                    // the film's second half step with the merged H/M pass
                    // (one launch on wide grids, as in stepping)
                    p.films = tvar(tp, m, V_P2);
                    CK(launch_hbulk_film<T>(p, nblk, 1, st));
                } else {
                    p.films = tvar(tp, m, V_C);
                    CK(launch_commit<T>(p, nblk, st));
                    CK(launch_hbulk<T>(p, 1, 1, st));
                }
            }
            return MPX_OK;
        };
        std::function<int(int, int)> rev;
        // the lambda psiH set a segment's reverse steps end in
        auto rev_end = [&](int len, int cs) { return merge ? cs ^ ((len + 1) & 1) : cs; };
        // one captured graph per kind serves every full-length segment
        auto run = [&](int kind, int len) -> mpx_status {
            auto direct = [&]() -> mpx_status {
                if (kind >= 2) return rev(len, kind - 2) < 0 ? MPX_E_DEVICE : MPX_OK;
                return fwd(len, kind == 0);
            };
            if (len != K || ncp < 2 || s->graph_steps <= 0) return direct();
            if (!gexec[kind]) {
                CK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                const mpx_status e1 = direct();
                hipGraph_t gg = nullptr;
                const hipError_t e2 = hipStreamEndCapture(st, &gg);
                if (e1 != MPX_OK) {
                    if (gg) (void)hipGraphDestroy(gg);
                    return e1;
                }
                CK(e2);
                graph[kind] = gg;
                CK(hipGraphInstantiate(&gexec[kind], gg, nullptr, nullptr, 0));
            }
            CK(hipGraphLaunch(gexec[kind], st));
            return MPX_OK;
        };

        // forward: the loss through a temporary probe (film energy, or the
        // weighted E component)
        {
            ProbeHost ph{};
            if (floss) {
                ph.dev.kind = MPX_PROBE_FILM_ENERGY;
                ph.dev.film = film;
                ph.dev.npart = ((long long)LF.cb[3] * LF.cb[4] * LF.cb[5] + 255) / 256;
            } else {
                ph.dev.kind = MPX_PROBE_FIELD;
                ph.dev.field = ls.field;
                ph.dev.i = ls.ijk[0];
                ph.dev.j = ls.ijk[1];
                ph.dev.k = ls.ijk[2];
            }
            ph.dev.nval = 1;
            ph.dev.cap = N;
            ph.dev.start = s->step;
            CK(hipMalloc(&ph.dev.data, N * sizeof(double)));
            if (ph.dev.npart) CK(hipMalloc(&ph.dev.part, ph.dev.npart * sizeof(double)));
            s->probes.push_back(ph);
            probe_added = true;
            drop_graph(s);
            if ((q = upload_probes(s)) != MPX_OK) return q;
        }
        std::vector<long long> pstep(ncp, 0);
        for (int g = 0; g < ncp; g++) {
            const long long c0 = (long long)g * K, len = std::min<long long>(K, N - c0);
            if (g < g0) {
                CK(launch_copy_segs(tab(g, 0), ns, L.nblk, st));
                cp[g].step = s->step;
                if ((q = enqueue_steps<T>(s, len)) != MPX_OK) return q;
                s->step += len;
                continue;
            }
            // a segment that keeps its tape: its magnetisation starts in the
            // tape's first slot and ends in slot len, from where it goes back
            // to the handle and to the next segment's first slot
            if (g == g0)
                for (int f = 0; f < nf; f++)
                    CK(hipMemcpyAsync(mslot(f, 0), s->films[f].M, mbytes(f), hipMemcpyDeviceToDevice, st));
            pstep[g] = s->step;
            if ((q = run(0, (int)len)) != MPX_OK) return q;
            s->step += len;
            CK(hipMemcpyAsync(pages + (size_t)(g - g0) * tp.bytes, tp.buf, tp.bytes, hipMemcpyDeviceToDevice, st));
            for (int f = 0; f < nf; f++) {
                CK(hipMemcpyAsync(s->films[f].M, mslot(f, (int)len), mbytes(f), hipMemcpyDeviceToDevice, st));
                CK(hipMemcpyAsync(mslot(f, 0), mslot(f, (int)len), mbytes(f), hipMemcpyDeviceToDevice, st));
            }
        }
        CK(launch_copy_segs(tab(g0, 0), ns, L.nblk, st));
        fin.step = s->step;
        std::vector<double> tr(N);
        CK(hipMemcpyAsync(tr.data(), s->probes.back().dev.data, N * sizeof(double), hipMemcpyDeviceToHost, st));
        CK(hipStreamSynchronize(st));
        {
            ProbeHost ph = s->probes.back();
            s->probes.pop_back();
            probe_added = false;
            (void)hipFree(ph.dev.data);
            (void)hipFree(ph.dev.part);
            drop_graph(s);
            if ((q = upload_probes(s)) != MPX_OK) return q;
        }
        // the seed is scaled by a power of two near 1/L (see the plain
        // schedule; for a weighted trace, near 1 / sum |w_i E_i|); exact in
        // float64
        double S = 1.0, mag = 0.0;
        if (floss) {
            double Lsum = 0.0;
            for (long long i = loss_from; i < N; i++) Lsum += tr[i];
            *loss = dt * Lsum;
            mag = *loss;
        } else {
            double Lsum = 0.0;
            for (long long i = 0; i < N; i++) {
                Lsum += ls.w[i] * tr[i];
                mag += std::fabs(ls.w[i] * tr[i]);
            }
            *loss = Lsum;
        }
        if (std::isfinite(mag) && mag > 0.0) S = std::ldexp(1.0, -std::ilogb(mag));

        // the loss term of the final state
        long long pw_slot = -1;
        if (floss) {
            AdjParams<T> A;
            adj_params<T>(s, h, A);
            CK(launch_tape_loss<T>(A.p, film, 0, tp.lossp(0), st, LF.cb));
            CK(launch_adj_loss_tape<T>(A, film, dt * S, tp.lossp(0), nullptr, 0, loss_from, st, LF.cb));
            if (d_lacc) {
                KParams<T> pe;
                fill_params<T>(s, pe, MODE_INPLACE, s->parity);
                CK(launch_adj_loss_eps_tape<T>(pe, film, dt * S, tp.lossp(0), nullptr, 0, loss_from, d_lacc, st,
                                               LF.cb));
            }
        } else {
            pw_slot = (long long)ls.ijk[0] + (long long)s->px * ((long long)ls.ijk[1] + (long long)s->n[1] * ls.ijk[2]);
            CK(hipMalloc(&d_w, N * sizeof(double)));
            CK(hipMemcpyAsync(d_w, ls.w, N * sizeof(double), hipMemcpyHostToDevice, st));
            CK(launch_add_one<T>((T *)h.lE[ls.field], pw_slot, S * ls.w[N - 1], st));
        }

        // the reverse steps' parameters for step m of the segment in hand
        auto params = [&](int m) {
            AdjParams<T> A;
            adj_params<T>(s, h, A);
            A.aflags = h.d_aflags;
            A.seg0 = h.d_seg0;
            A.m = m;
            A.btape = neps > 0 ? tp.boxp(m) : nullptr;
            A.gca_box = h.gbox_a;
            A.gcb_box = h.gbox_b;
            for (int a = 0; a < 3; a++) {
                A.bb[a] = eps_box[a];
                A.bs[a] = eps_box[3 + a];
            }
            A.ltape = floss ? tp.lossp(m) : nullptr;
            A.lfilm = film;
            A.lscale = dt * S;
            A.loss_from = loss_from;
            A.pw = d_w;
            A.pw_slot = pw_slot;
            A.pw_comp = ls.field;
            A.pw_scale = S;
            for (int c = 0; c < 3; c++) {
                A.mu[c] = (T *)h.mu[c];
                for (int a = 0; a < 3; a++) A.lpsiE2[c][a] = (T *)h.lpsiE2[c][a];
            }
            return A;
        };
        // lambda psiH: set 0 (adj_params' lpsiH) or 1 (lpsiH2); a half-step
        // pass reads set `from` and writes the other
        auto psi_sets = [&](AdjParams<T> &A, int from) {
            for (int c = 0; c < 3; c++)
                for (int a = 0; a < 3; a++) {
                    A.lpsiH[c][a] = (T *)(from ? h.lpsiH2[c][a] : h.lpsiH[c][a]);
                    A.lpsiHo[c][a] = (T *)(from ? h.lpsiH[c][a] : h.lpsiH2[c][a]);
                }
        };
        auto loss_eps = [&](int m) -> mpx_status {
            if (d_lacc) {
                // the loss's eps_r term of the step's input state
                KParams<T> pe;
                fill_params<T>(s, pe, MODE_INPLACE, s->parity);
                CK(launch_adj_loss_eps_tape<T>(pe, film, dt * S, tp.lossp(m), h.d_seg0, m, loss_from, d_lacc, st,
                                               LF.cb));
            }
            return MPX_OK;
        };
        // the adjoint steps of a segment from its tape, lambda psiH starting
        // in set cs; returns the set it ends in.  Per step m (backwards): the
        // second half step's transpose, the E step's, the first half step's.
        // With `merge`, the first half step of step m and the second of step
        // m - 1 share one field pass (their film parts run before it).
        rev = [&](int len, int cs) -> int {
            int cur = cs;
            for (int m = len - 1; m >= 0; m--) {
                if (!merge || m == len - 1) {
                    if (loss_eps(m) != MPX_OK) return -1;
                    AdjParams<T> A = params(m);
                    psi_sets(A, cur);
                    A.p.films = tvar(tp, m, V_P1);
                    A.af = h.d_af;
                    if (launch_adj_half_fused<T>(A, nblk, 0, h.film_nr.data(), st) != hipSuccess) return -1;
                    cur ^= 1;
                    if (launch_adj_estep_fused<T>(A, st) != hipSuccess) return -1;
                }
                if (merge && m > 0) {
                    // the first half step of step m: its film part, the loss
                    // term's lambda H part of step m's input state
                    AdjParams<T> A = params(m);
                    psi_sets(A, cur);
                    A.p.films = tvar(tp, m, V_R1);
                    A.af = h.d_af2;
                    if (launch_adj_film_part<T>(A, nblk, h.film_nr.data(), st) != hipSuccess) return -1;
                    if (floss && launch_adj_loss_h<T>(A, LF.cb, st) != hipSuccess) return -1;
                    // the second half step of step m - 1: its film part
                    if (loss_eps(m - 1) != MPX_OK) return -1;
                    AdjParams<T> B = params(m - 1);
                    psi_sets(B, cur ^ 1);
                    B.p.films = tvar(tp, m - 1, V_P1);
                    B.af = h.d_af;
                    if (launch_adj_film_part<T>(B, nblk, h.film_nr.data(), st) != hipSuccess) return -1;
                    // both field transposes in one pass, then step m - 1's E step
                    A.afb = h.d_af;
                    if (launch_adj_hfield2<T>(A, st) != hipSuccess) return -1;
                    cur ^= 1;
                    if (launch_adj_estep_fused<T>(B, st) != hipSuccess) return -1;
                } else {
                    // the first half step (with the E step's lambda E = ca
                    // lambda E', the eps-box sums and the loss term of the
                    // step's input state)
                    AdjParams<T> A = params(m);
                    psi_sets(A, cur);
                    A.p.films = tvar(tp, m, V_R1);
                    A.af = h.d_af2;
                    if (launch_adj_half_fused<T>(A, nblk, 1, h.film_nr.data(), st) != hipSuccess) return -1;
                    cur ^= 1;
                }
            }
            return cur;
        };
        int psi_cur = 0;
        for (int g = ncp - 1; g >= 0; g--) {
            const long long c0 = (long long)g * K;
            const int len = (int)std::min<long long>(K, N - c0);
            if (g >= g0) {
                CK(hipMemcpyAsync(tp.buf, pages + (size_t)(g - g0) * tp.bytes, tp.bytes, hipMemcpyDeviceToDevice,
                                  st));
                s->step = pstep[g];
            } else {
                CK(launch_copy_segs(tab(g, 2), ns, L.nblk, st));
                s->step = cp[g].step;
            }
            CK(launch_set_step(s->d_step, s->step, st));
            CK(launch_set_step(h.d_seg0, c0, st));
            if (g < g0 && (q = run(1, len)) != MPX_OK) return q;
            if ((q = run(2 + psi_cur, len)) != MPX_OK) return q;
            psi_cur = rev_end(len, psi_cur);
        }
        // the initial magnetisation M0 = Ms u
        if (step0 == 0 && s->have_u) CK(launch_adj_init_ms(s->d_blocktab, nblk, s->d_films, h.d_af, s->u, st));
        if (neps > 0) {
            KParams<T> p;
            fill_params<T>(s, p, MODE_INPLACE, s->parity);
            CK(launch_adj_eps_box<T>(p, eps_box, h.gbox_a, h.gbox_b, h.d_out, st));
            CK(hipMemcpyAsync(geps, h.d_out, neps * sizeof(double), hipMemcpyDeviceToHost, st));
        }
        CK(hipStreamSynchronize(st));
        if (d_lacc && (q = add_loss_eps(s, d_lacc, LF.cb, eps_box, geps)) != MPX_OK) return q;
        for (long long t = 0; t < neps; t++) geps[t] /= S;
        if ((q = film_grads(s, h, S, ms_box, gH0, gms)) != MPX_OK) return q;
        // leave the handle at the end of the forward run
        CK(launch_copy_segs(tab(g0, 1), ns, L.nblk, st));
        s->step = fin.step;
        CK(launch_set_step(s->d_step, fin.step, st));
        CK(hipStreamSynchronize(st));
        return MPX_OK;
    };
    mpx_status r = body();
    if (probe_added) {
        ProbeHost ph = s->probes.back();
        s->probes.pop_back();
        (void)hipFree(ph.dev.data);
        (void)hipFree(ph.dev.part);
        drop_graph(s);
        (void)upload_probes(s);
    }
    if (r != MPX_OK) (void)hipStreamSynchronize(st);
    (void)hipFree(d_w);
    (void)hipFree(d_lacc);
    for (int k = 0; k < 4; k++) {
        if (gexec[k]) (void)hipGraphExecDestroy(gexec[k]);
        if (graph[k]) (void)hipGraphDestroy(graph[k]);
    }
    (void)hipFree(pages);
    s->fused = saved_fused;
    adj_free(h);
    tape_free(tp);
    for (auto &z : cp) (void)hipFree(z.buf);
    (void)hipFree(fin.buf);
    return r;
}

} // namespace

// ---------------------------------------------------------------------------
// Scratch of the no-allocation energy call: a static device array (each GPU
// the library runs on holds its own copy until the process ends).  In host
// code `energy_scratch` names a host-side stand-in, never a device address:
// the device address is taken once per device with hipGetSymbolAddress and
// used everywhere instead.  Layout: the three sums at 0, the per-block
// partial pairs from kScratchPart on.
// ---------------------------------------------------------------------------
namespace {
constexpr long long kScratchDoubles = 1LL << 21; // 16 MiB per device
constexpr long long kScratchPart = 32;           // 256-byte offset of the partials
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_dev[kScratchDevices] = {};
} // namespace

static __device__ __align__(256) double energy_scratch[kScratchDoubles];

__global__ void k_clear3(double *p) {
    if (threadIdx.x < 3) p[threadIdx.x] = 0.0;
}

namespace {
// the device address of this device's scratch (the handle's device current)
mpx_status energy_scratch_ptr(mpx_sim *s, double **out) {
    if (s->device < 0 || s->device >= kScratchDevices) return fail(s, MPX_E_UNSUPPORTED, "device index too large");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[s->device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(energy_scratch));
        if (e != hipSuccess || !ptr) return dev_fail(s, e != hipSuccess ? e : hipErrorInvalidSymbol,
                                                     "hipGetSymbolAddress(energy_scratch)");
        g_scratch_dev[s->device] = (double *)ptr;
    }
    *out = g_scratch_dev[s->device];
    return MPX_OK;
}
} // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

uint32_t mpx_abi_version(void) { return MPX_ABI_VERSION; }

mpx_status mpx_create(const mpx_grid_desc *g, mpx_precision prec, int32_t hip_device, void *hip_stream,
                      mpx_sim **out) {
    if (!g || !out) return MPX_E_INVALID;
    *out = nullptr;
    if (g->nx < 1 || g->ny < 1 || g->nz < 1 || !(g->dx > 0) || !(g->dy > 0) || !(g->dz > 0)) return MPX_E_INVALID;
    if (prec != MPX_F64 && prec != MPX_F32) return MPX_E_INVALID;
    const int nn[3] = {g->nx, g->ny, g->nz};
    for (int a = 0; a < 3; a++) {
        const int lo = g->bc[2 * a], hi = g->bc[2 * a + 1];
        if (lo < 0 || lo > 2 || hi < 0 || hi > 2) return MPX_E_INVALID;
        if ((lo == MPX_BC_PERIODIC) != (hi == MPX_BC_PERIODIC)) return MPX_E_INVALID;
        const int plo = lo == MPX_BC_PML ? g->pml_cells[2 * a] : 0;
        const int phi = hi == MPX_BC_PML ? g->pml_cells[2 * a + 1] : 0;
        if (plo < 0 || phi < 0 || (lo == MPX_BC_PML && plo < 1) || (hi == MPX_BC_PML && phi < 1)) return MPX_E_INVALID;
        if (plo + phi >= nn[a]) return MPX_E_INVALID;
    }
    // the stability limit of the 3-D Yee scheme
    const double dt_max = 1.0 / (C0 * std::sqrt(1.0 / (g->dx * g->dx) + 1.0 / (g->dy * g->dy) + 1.0 / (g->dz * g->dz)));
    double dt = g->dt;
    if (!(dt > 0)) {
        if (!(g->courant > 0) || g->courant > 1.0) return MPX_E_INVALID;
        dt = g->courant * dt_max;
    } else if (!(dt <= dt_max) || !std::isfinite(dt)) {
        return MPX_E_INVALID; // an explicit step above the limit would grow without bound
    }
    mpx_sim *s = new mpx_sim();
    s->g = *g;
    s->prec = prec;
    s->device = hip_device;
    s->esz = prec == MPX_F64 ? 8 : 4;
    for (int a = 0; a < 3; a++) {
        s->n[a] = nn[a];
        s->per[a] = g->bc[2 * a] == MPX_BC_PERIODIC;
        s->nlo[a] = g->bc[2 * a] == MPX_BC_PML ? g->pml_cells[2 * a] : 0;
        s->nhi[a] = g->bc[2 * a + 1] == MPX_BC_PML ? g->pml_cells[2 * a + 1] : 0;
        if (s->nlo[a] || s->nhi[a]) s->any_pml = true;
    }
    s->d[0] = g->dx;
    s->d[1] = g->dy;
    s->d[2] = g->dz;
    s->dt = dt;
    s->px = (g->nx + 31) / 32 * 32;
    s->nslot = (long long)s->px * g->ny * g->nz;
    hipError_t e = hipSetDevice(hip_device);
    if (e != hipSuccess) {
        delete s;
        return MPX_E_DEVICE;
    }
    mpx_status r = MPX_OK;
    auto setup = [&]() -> mpx_status {
        if (hip_stream) {
            s->stream = (hipStream_t)hip_stream;
        } else {
            CK(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
            s->own_stream = true;
        }
        for (int c = 0; c < 3; c++) {
            CK(hipMalloc(&s->E[c], s->nslot * s->esz));
            CK(hipMalloc(&s->H[c], s->nslot * s->esz));
            CK(hipMalloc(&s->E2[c], s->nslot * s->esz));
            CK(hipMalloc(&s->H2[c], s->nslot * s->esz));
            CK(hipMemset(s->E[c], 0, s->nslot * s->esz));
            CK(hipMemset(s->H[c], 0, s->nslot * s->esz));
            CK(hipMemset(s->E2[c], 0, s->nslot * s->esz));
            CK(hipMemset(s->H2[c], 0, s->nslot * s->esz));
        }
        CK(hipMalloc(&s->d_coef, kCoefEntries * (prec == MPX_F64 ? sizeof(CoefDev<double>) : sizeof(CoefDev<float>))));
        {
            const size_t vb = 256 * (prec == MPX_F64 ? kCoefRow<double> * sizeof(double) : kCoefRow<float> * sizeof(float));
            CK(hipMalloc(&s->d_coefv, vb));
            CK(hipMemset(s->d_coefv, 0, vb));
        }
        CK(hipMalloc(&s->d_id, s->nslot));
        CK(hipMemset(s->d_id, 0, s->nslot));
        CK(hipMalloc(&s->d_cls, s->nslot));
        CK(hipMemset(s->d_cls, 0, s->nslot));
        CK(hipMalloc(&s->d_mat, 256 * sizeof(MatDev)));
        CK(hipMemset(s->d_mat, 0, 256 * sizeof(MatDev)));
        CK(hipMalloc(&s->d_step, sizeof(long long)));
        CK(hipMemset(s->d_step, 0, sizeof(long long)));
        CK(hipMalloc(&s->d_flag, sizeof(int)));
        CK(hipMemset(s->d_flag, 0, sizeof(int)));
        return prec == MPX_F64 ? upload_profiles<double>(s) : upload_profiles<float>(s);
    };
    r = setup();
    if (r != MPX_OK) {
        mpx_destroy(s);
        return r == MPX_E_DEVICE ? MPX_E_NOMEM : r;
    }
    *out = s;
    return MPX_OK;
}

mpx_status mpx_destroy(mpx_sim *s) {
    if (!s) return MPX_OK;
    (void)hipSetDevice(s->device);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    drop_graph(s);
    for (auto e : s->ev) (void)hipEventDestroy(e);
    (void)hipFree(s->d_coef);
    (void)hipFree(s->d_coefv);
    for (int c = 0; c < 3; c++) {
        (void)hipFree(s->E[c]);
        (void)hipFree(s->H[c]);
        (void)hipFree(s->E2[c]);
        (void)hipFree(s->H2[c]);
        (void)hipFree(s->bE[c]);
        (void)hipFree(s->cE[c]);
        (void)hipFree(s->bH[c]);
        (void)hipFree(s->cH[c]);
        for (int w = 0; w < 3; w++) {
            (void)hipFree(s->psiE[c][w]);
            (void)hipFree(s->psiE2[c][w]);
            (void)hipFree(s->psiH[c][w]);
        }
    }
    free_films(s);
    for (auto &src : s->srcs) (void)hipFree(src.table);
    for (auto &pr : s->probes) {
        (void)hipFree(pr.dev.data);
        (void)hipFree(pr.dev.part);
    }
    (void)hipFree(s->d_probes);
    (void)hipFree(s->d_srcs);
    (void)hipFree(s->d_pflags);
    (void)hipFree(s->d_pflags_w);
    (void)hipFree(s->d_mixed);
    (void)hipFree(s->d_cls16);
    (void)hipFree(s->d_id);
    (void)hipFree(s->d_cls);
    (void)hipFree(s->d_mat);
    (void)hipFree(s->d_step);
    (void)hipFree(s->d_flag);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
    return MPX_OK;
}

mpx_status mpx_query_field(const mpx_sim *s, int32_t field, int64_t dims[4], int64_t *bytes) {
    if (!s || !dims || field < 0 || field > 11) return MPX_E_INVALID;
    const int f = field < 6 ? field : 3 + (field - 6) % 3;
    for (int a = 0; a < 3; a++) dims[a] = natural_dim(s, f, a);
    dims[3] = field < 6 ? 1 : 3;
    const size_t esz = field < 6 ? s->esz : 8;
    if (bytes) *bytes = dims[0] * dims[1] * dims[2] * dims[3] * (int64_t)esz;
    return MPX_OK;
}

mpx_status mpx_set_materials(mpx_sim *s, const mpx_material *table, int32_t n, const uint8_t *cell_ids) {
    mpx_status r = check_live(s);
    if (r != MPX_OK) return r;
    if (!table || !cell_ids || n < 1 || n > 256) return fail(s, MPX_E_INVALID, "bad material table");
    // a film probe names a film of the current material map (its index and
    // partial-sum layout were checked against that map's films)
    for (auto &ph : s->probes)
        if (ph.dev.kind == MPX_PROBE_MEAN_M || ph.dev.kind == MPX_PROBE_FILM_ENERGY)
            return fail(s, MPX_E_STATE, "film probes exist: set the materials before adding film probes");
    const long long ncell = (long long)s->n[0] * s->n[1] * s->n[2];
    for (long long q = 0; q < ncell; q++)
        if (cell_ids[q] >= n) return fail(s, MPX_E_INVALID, "cell id outside the material table");
    std::vector<mpx_material> mats(table, table + n);
    std::vector<uint8_t> ids(cell_ids, cell_ids + ncell);
    // a magnetic cell may not sit in, or next to, a PML slab
    for (int k = 0; k < s->n[2]; k++)
        for (int j = 0; j < s->n[1]; j++)
            for (int i = 0; i < s->n[0]; i++) {
                if (!(mats[ids[i + (size_t)s->n[0] * (j + (size_t)s->n[1] * k)]].Ms > 0)) continue;
                const int c3[3] = {i, j, k};
                for (int a = 0; a < 3; a++)
                    for (int dd = -1; dd <= 1; dd++) {
                        const int x = c3[a] + dd;
                        if (x < 0 || x >= s->n[a]) continue;
                        if (in_pml_cell(s, a, x)) return fail(s, MPX_E_INVALID, "magnetic cell in or next to a PML");
                    }
            }
    s->mats = mats;
    s->ids = ids;
    std::vector<FilmHost> films = discover_films(s);
    if ((int)films.size() > kMaxFilms) return fail(s, MPX_E_INVALID, "more than 64 films");
    for (auto &f : films) {
        for (int a = 0; a < 3; a++) {
            const int lo = f.cb[a], nn = f.cb[3 + a];
            if (s->per[a] && nn == s->n[a]) {
                f.b0[a] = 0;
                f.bn[a] = s->n[a];
            } else if (lo >= 1 && lo + nn + 1 <= s->n[a]) {
                f.b0[a] = lo;
                f.bn[a] = nn + 1;
            } else {
                s->have_mat = false;
                return fail(s, MPX_E_UNSUPPORTED, "film touches a domain face (keep one cell of gap)");
            }
        }
        f.ns = (long long)f.bn[0] * f.bn[1] * f.bn[2];
    }
    drop_graph(s);
    free_films(s);
    s->films = films;
    // device copies
    std::vector<MatDev> md(256);
    memset(md.data(), 0, md.size() * sizeof(MatDev));
    for (int q = 0; q < n; q++) {
        md[q].eps_r = mats[q].eps_r;
        md[q].sigma = mats[q].sigma;
        md[q].Ms = mats[q].Ms;
        md[q].alpha = mats[q].alpha;
        md[q].gamma_abs = mats[q].gamma_abs;
        md[q].is_pec = mats[q].is_pec ? 1 : 0;
    }
    CK(hipMemcpy(s->d_mat, md.data(), 256 * sizeof(MatDev), hipMemcpyHostToDevice));
    // edge coefficients from the four cells around an edge, in the device's
    // order and operations (sum of four in order, mean, ca, cb); a PEC edge
    // stays zero
    auto coef_of = [&](const int *m4) {
        CoefDev<double> c{};
        double se = 0.0, ss = 0.0;
        bool pec = false;
        for (int r4 = 0; r4 < 4; r4++) {
            se += mats[m4[r4]].eps_r;
            ss += mats[m4[r4]].sigma;
            pec = pec || mats[m4[r4]].is_pec;
        }
        const double eps = EPS0 * (se / 4);
        const double sig = ss / 4;
        const double den = sig / 2.0 + eps / s->dt;
        c.ca = -(sig / 2.0 - eps / s->dt) / den;
        c.cb = 1.0 / den;
        c.pec = pec ? 1 : 0;
        if (pec) c.ca = c.cb = 0.0;
        return c;
    };
    std::vector<CoefDev<double>> cd(kCoefEntries);
    memset(cd.data(), 0, cd.size() * sizeof(cd[0]));
    for (int q = 0; q < n; q++) {
        const int m4[4] = {q, q, q, q};
        const CoefDev<double> c = coef_of(m4);
        for (int C = 0; C < kCoefPerClass; C++) cd[kCoefPerClass * q + C] = c;
    }
    std::vector<uint8_t> slots(s->nslot, 0);
    for (int k = 0; k < s->n[2]; k++)
        for (int j = 0; j < s->n[1]; j++)
            memcpy(&slots[(size_t)s->px * (j + (size_t)s->n[1] * k)], &ids[(size_t)s->n[0] * (j + (size_t)s->n[1] * k)],
                   s->n[0]);
    CK(hipMemcpy(s->d_id, slots.data(), s->nslot, hipMemcpyHostToDevice));
    CK(launch_classify(s->d_id, s->d_cls, s->n, s->per, s->px, s->stream));
    {
        // compound classes: the distinct triples of edge coefficients among
        // the slots the classifier left mixed, most frequent first (ties in
        // key order), get the class ids from n up to 254; their slots then
        // take the table path, the others keep the general one
        std::vector<uint8_t> hc(s->nslot);
        CK(hipMemcpyAsync(hc.data(), s->d_cls, s->nslot, hipMemcpyDeviceToHost, s->stream));
        CK(hipStreamSynchronize(s->stream));
        // per mixed slot, the ids of the four cells of each edge (a wall
        // edge, never updated, as a flag) key a first table; the edge
        // coefficients are computed once per distinct id key, and id keys
        // with equal coefficient triples share a class
        struct IdKey {
            unsigned long long lo = 0, hi = 0; // 12 ids, then the wall flags
            bool operator==(const IdKey &o) const { return lo == o.lo && hi == o.hi; }
        };
        struct IdKeyHash {
            size_t operator()(const IdKey &k) const {
                return (size_t)(k.lo * 0x9e3779b97f4a7c15ULL ^ (k.hi + 0x632be59bd9b4e019ULL) * 0xbf58476d1ce4e5b9ULL);
            }
        };
        std::unordered_map<IdKey, int, IdKeyHash> id_index;
        std::vector<IdKey> id_keys;
        std::vector<long long> id_count;
        std::vector<std::pair<long long, int>> slot_key; // mixed slot -> its id key
        for (int k = 0; k < s->n[2]; k++)
            for (int j = 0; j < s->n[1]; j++)
                for (int i = 0; i < s->n[0]; i++) {
                    const long long q = (long long)i + (long long)s->px * ((long long)j + (long long)s->n[1] * k);
                    if (hc[q] != kMixed) continue;
                    const int idx[3] = {i, j, k};
                    uint8_t m12[12] = {};
                    unsigned wall_bits = 0;
                    for (int C = 0; C < 3; C++) {
                        bool wall = false;
                        for (int a = 0; a < 3; a++)
                            if (a != C && !s->per[a] && idx[a] == 0) wall = true;
                        if (wall) {
                            wall_bits |= 1u << C;
                            continue;
                        }
                        const int C1 = (C + 1) % 3, C2 = (C + 2) % 3;
                        for (int u = 0; u < 2; u++)
                            for (int v = 0; v < 2; v++) {
                                int cc[3] = {i, j, k};
                                cc[C1] -= 1 - u;
                                cc[C2] -= 1 - v;
                                for (int a = 0; a < 3; a++)
                                    if (cc[a] < 0) cc[a] += s->n[a]; // periodic (walls excluded above)
                                m12[4 * C + 2 * u + v] =
                                    ids[(size_t)cc[0] + (size_t)s->n[0] * (cc[1] + (size_t)s->n[1] * cc[2])];
                            }
                    }
                    IdKey key;
                    memcpy(&key.lo, m12, 8);
                    unsigned tail = 0;
                    memcpy(&tail, m12 + 8, 4);
                    key.hi = (unsigned long long)tail | ((unsigned long long)wall_bits << 32);
                    auto it = id_index.find(key);
                    int ki;
                    if (it == id_index.end()) {
                        ki = (int)id_keys.size();
                        id_index.emplace(key, ki);
                        id_keys.push_back(key);
                        id_count.push_back(0);
                    } else {
                        ki = it->second;
                    }
                    id_count[ki]++;
                    slot_key.emplace_back(q, ki);
                }
        // the coefficient triple of each id key, merged by value
        using Key = std::array<unsigned long long, 9>;
        struct Entry {
            long long count = 0;
            int cls = kMixed;
            CoefDev<double> e[3];
        };
        std::map<Key, Entry> seen;
        std::vector<Entry *> entry_of(id_keys.size(), nullptr);
        for (size_t ki = 0; ki < id_keys.size(); ki++) {
            uint8_t m12[12];
            memcpy(m12, &id_keys[ki].lo, 8);
            const unsigned tail = (unsigned)(id_keys[ki].hi & 0xffffffffULL);
            memcpy(m12 + 8, &tail, 4);
            const unsigned wall_bits = (unsigned)(id_keys[ki].hi >> 32);
            CoefDev<double> e[3];
            Key key{};
            for (int C = 0; C < 3; C++) {
                if (wall_bits & (1u << C)) {
                    e[C] = CoefDev<double>{};
                    e[C].pec = 1;
                } else {
                    const int m4[4] = {m12[4 * C], m12[4 * C + 1], m12[4 * C + 2], m12[4 * C + 3]};
                    e[C] = coef_of(m4);
                }
                memcpy(&key[3 * C], &e[C].ca, 8);
                memcpy(&key[3 * C + 1], &e[C].cb, 8);
                key[3 * C + 2] = (unsigned long long)e[C].pec;
            }
            auto it = seen.find(key);
            if (it == seen.end()) {
                it = seen.emplace(key, Entry{}).first;
                for (int C = 0; C < 3; C++) it->second.e[C] = e[C];
            }
            it->second.count += id_count[ki];
            entry_of[ki] = &it->second; // map nodes are stable
        }
        std::vector<std::pair<long long, Entry *>> order;
        for (auto &kv : seen) order.emplace_back(kv.second.count, &kv.second);
        std::stable_sort(order.begin(), order.end(),
                         [](const std::pair<long long, Entry *> &a, const std::pair<long long, Entry *> &b) {
                             return a.first > b.first;
                         });
        int next = n;
        for (auto &o : order) {
            if (next >= kMixed) break; // table full: the rest keep the mixed path
            o.second->cls = next;
            for (int C = 0; C < 3; C++) cd[kCoefPerClass * next + C] = o.second->e[C];
            next++;
        }
        // the triples left without a class get an entry of the extended
        // table (up to kMaxExt of them; beyond, the cell-id path)
        constexpr long long kMaxExt = 1 << 20;
        std::vector<CoefDev<double>> cdx;
        std::map<const Entry *, int> ext_of;
        for (auto &o : order) {
            if (o.second->cls != kMixed || (long long)ext_of.size() >= kMaxExt) continue;
            ext_of.emplace(o.second, (int)ext_of.size());
            for (int C = 0; C < 3; C++) cdx.push_back(o.second->e[C]);
        }
        // when the extended table has entries: a 16-bit class per slot for
        // the E pass, the class byte's value where it is below 255 and
        // otherwise 256 + the triple's index in the extended table (the
        // table's rows after the 256 classes'), for the 65279 most frequent
        // extended triples; the slots of the rarer ones (and of triples
        // beyond the extended table) take 0xffff and go on the mixed list,
        // in slot order, with their extended index (or -1: the cell-id path)
        constexpr int kMaxCls16 = 0xffff - 256;
        std::vector<int4> mixed;
        std::vector<uint16_t> c16;
        if (!ext_of.empty()) {
            c16.resize(s->nslot);
            for (long long q = 0; q < s->nslot; q++) c16[q] = hc[q];
        }
        bool changed = false;
        for (auto &sk : slot_key) {
            const Entry *en = entry_of[sk.second];
            const long long q = sk.first;
            if (en->cls == kMixed) {
                auto it = ext_of.find(en);
                const int e = it == ext_of.end() ? -1 : it->second;
                if (e >= 0 && e < kMaxCls16) {
                    c16[q] = (uint16_t)(256 + e);
                } else {
                    if (!c16.empty()) c16[q] = 0xffff;
                    mixed.push_back(make_int4((int)(q % s->px), (int)((q / s->px) % s->n[1]),
                                              (int)(q / ((long long)s->px * s->n[1])), e));
                }
                continue;
            }
            hc[q] = (uint8_t)en->cls;
            if (!c16.empty()) c16[q] = (uint16_t)en->cls;
            changed = true;
        }
        if (changed) CK(hipMemcpy(s->d_cls, hc.data(), s->nslot, hipMemcpyHostToDevice));
        (void)hipFree(s->d_cls16);
        s->d_cls16 = nullptr;
        if (!c16.empty()) {
            CK(hipMalloc(&s->d_cls16, c16.size() * sizeof(uint16_t)));
            CK(hipMemcpy(s->d_cls16, c16.data(), c16.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
        }
        (void)hipFree(s->d_mixed);
        s->d_mixed = nullptr;
        CK(hipMalloc(&s->d_mixed, std::max<size_t>(1, mixed.size()) * sizeof(int4)));
        if (!mixed.empty())
            CK(hipMemcpy(s->d_mixed, mixed.data(), mixed.size() * sizeof(int4), hipMemcpyHostToDevice));
        s->nmixed = (int)mixed.size();
        // one table: the classes' entries, then the extended entries (the E
        // pass indexes an extended triple as class 256 + its index)
        const size_t ntot = (size_t)kCoefEntries + cdx.size();
        (void)hipFree(s->d_coef);
        s->d_coef = nullptr;
        s->n_coef_ext = (long long)cdx.size() / kCoefPerClass;
        // the packed rows: ca, cb of the x, y, z edges of each row, in the
        // field precision (float: rounded once from the float64 values, as
        // in the table)
        {
            const size_t nrow = ntot / kCoefPerClass;
            const int rw = s->prec == MPX_F64 ? kCoefRow<double> : kCoefRow<float>;
            std::vector<double> v64((size_t)nrow * rw, 0.0);
            for (size_t r = 0; r < nrow; r++)
                for (int C = 0; C < kCoefPerClass; C++) {
                    const size_t q = r * kCoefPerClass + C;
                    const CoefDev<double> &c = q < (size_t)kCoefEntries ? cd[q] : cdx[q - kCoefEntries];
                    v64[r * rw + 2 * C] = c.pec ? 0.0 : c.ca;
                    v64[r * rw + 2 * C + 1] = c.pec ? 0.0 : c.cb;
                }
            (void)hipFree(s->d_coefv);
            s->d_coefv = nullptr;
            if (s->prec == MPX_F64) {
                CK(hipMalloc(&s->d_coefv, v64.size() * sizeof(double)));
                CK(hipMemcpy(s->d_coefv, v64.data(), v64.size() * sizeof(double), hipMemcpyHostToDevice));
            } else {
                std::vector<float> v32(v64.size());
                for (size_t q = 0; q < v64.size(); q++) v32[q] = (float)v64[q];
                CK(hipMalloc(&s->d_coefv, v32.size() * sizeof(float)));
                CK(hipMemcpy(s->d_coefv, v32.data(), v32.size() * sizeof(float), hipMemcpyHostToDevice));
            }
        }
        if (s->prec == MPX_F64) {
            std::vector<CoefDev<double>> all(cd);
            all.insert(all.end(), cdx.begin(), cdx.end());
            CK(hipMalloc(&s->d_coef, ntot * sizeof(CoefDev<double>)));
            CK(hipMemcpy(s->d_coef, all.data(), ntot * sizeof(all[0]), hipMemcpyHostToDevice));
        } else {
            std::vector<CoefDev<float>> cf(ntot);
            memset(cf.data(), 0, cf.size() * sizeof(cf[0]));
            for (size_t q = 0; q < ntot; q++) {
                const CoefDev<double> &c = q < (size_t)kCoefEntries ? cd[q] : cdx[q - kCoefEntries];
                cf[q].ca = (float)c.ca;
                cf[q].cb = (float)c.cb;
                cf[q].pec = c.pec;
            }
            CK(hipMalloc(&s->d_coef, ntot * sizeof(CoefDev<float>)));
            CK(hipMemcpy(s->d_coef, cf.data(), ntot * sizeof(cf[0]), hipMemcpyHostToDevice));
        }
    }
    if ((r = update_pass_flags(s)) != MPX_OK) return r;
    std::vector<int4> bt, bte;
    std::vector<FilmDev> fd;
    for (int fi = 0; fi < (int)s->films.size(); fi++) {
        FilmHost &f = s->films[fi];
        CK(hipMalloc(&f.M, 9 * f.ns * sizeof(double)));
        CK(hipMalloc(&f.M1, 9 * f.ns * sizeof(double)));
        CK(hipMalloc(&f.H1, 3 * f.ns * sizeof(double)));
        CK(hipMemset(f.M, 0, 9 * f.ns * sizeof(double)));
        CK(hipMemset(f.M1, 0, 9 * f.ns * sizeof(double)));
        CK(hipMemset(f.H1, 0, 3 * f.ns * sizeof(double)));
        {
            // per-face Ms, alpha, |gamma| (the same means the kernels would form)
            std::vector<double> prm(9 * f.ns);
            for (int c = 0; c < 3; c++)
                for (long long l = 0; l < f.ns; l++) {
                    const int idx[3] = {f.b0[0] + (int)(l % f.bn[0]), f.b0[1] + (int)((l / f.bn[0]) % f.bn[1]),
                                        f.b0[2] + (int)(l / ((long long)f.bn[0] * f.bn[1]))};
                    double ms, al, ga;
                    site_params_h(s, c, idx, ms, al, ga);
                    prm[(c * 3 + 0) * f.ns + l] = ms;
                    prm[(c * 3 + 1) * f.ns + l] = al;
                    prm[(c * 3 + 2) * f.ns + l] = ga;
                }
            CK(hipMalloc(&f.prm, prm.size() * sizeof(double)));
            CK(hipMemcpy(f.prm, prm.data(), prm.size() * sizeof(double), hipMemcpyHostToDevice));
        }
        for (int c = 0; c < 3; c++) {
            f.blk0[c] = (int)bt.size();
            const long long tiles = (f.ns + 255) / 256;
            f.nblk[c] = (int)tiles;
            for (long long t = 0; t < tiles; t++) bt.push_back(make_int4(fi, c, (int)(t * 256), 0));
        }
        // face box grown by one layer on the low side of each non-spanned axis
        for (int a = 0; a < 3; a++) {
            const bool span = s->per[a] && f.bn[a] == s->n[a];
            f.e0[a] = span ? 0 : f.b0[a] - 1;
            f.en[a] = span ? s->n[a] : f.bn[a] + 1;
        }
        f.nse = (long long)f.en[0] * f.en[1] * f.en[2];
        // the kernels index a family's grown box with 32-bit integers
        if (f.nse >= (1ll << 31)) {
            s->have_mat = false;
            return fail(s, MPX_E_UNSUPPORTED, "film face box above 2^31 faces");
        }
        CK(hipMalloc(&f.Bn, 3 * f.nse * sizeof(double)));
        CK(hipMalloc(&f.Bs, 3 * f.nse * sizeof(double)));
        CK(hipMemset(f.Bn, 0, 3 * f.nse * sizeof(double)));
        CK(hipMemset(f.Bs, 0, 3 * f.nse * sizeof(double)));
        CK(hipMalloc(&f.Bn2, 3 * f.nse * sizeof(double)));
        CK(hipMalloc(&f.Bs2, 3 * f.nse * sizeof(double)));
        CK(hipMemset(f.Bn2, 0, 3 * f.nse * sizeof(double)));
        CK(hipMemset(f.Bs2, 0, 3 * f.nse * sizeof(double)));
        for (int c = 0; c < 3; c++)
            for (long long t = 0; t < (f.nse + 255) / 256; t++) bte.push_back(make_int4(fi, c, (int)(t * 256), 0));
        FilmDev d{};
        for (int a = 0; a < 3; a++) {
            d.b0[a] = f.b0[a];
            d.bn[a] = f.bn[a];
            d.blk0[a] = f.blk0[a];
            d.nblk[a] = f.nblk[a];
        }
        for (int a = 0; a < 6; a++) d.cb[a] = f.cb[a];
        d.ns = f.ns;
        d.ncells = (double)f.ncells;
        d.M = f.M;
        d.M1 = f.M1;
        d.H1 = f.H1;
        d.prm = f.prm;
        for (int a = 0; a < 3; a++) {
            d.e0[a] = f.e0[a];
            d.en[a] = f.en[a];
        }
        d.nse = f.nse;
        d.Bn = f.Bn;
        d.Bs = f.Bs;
        d.Bn2 = f.Bn2;
        d.Bs2 = f.Bs2;
        fd.push_back(d);
    }
    s->nblk = (int)bt.size();
    if (!fd.empty()) {
        CK(hipMalloc(&s->d_films, fd.size() * sizeof(FilmDev)));
        CK(hipMemcpy(s->d_films, fd.data(), fd.size() * sizeof(FilmDev), hipMemcpyHostToDevice));
        CK(hipMalloc(&s->d_blocktab, bt.size() * sizeof(int4)));
        CK(hipMemcpy(s->d_blocktab, bt.data(), bt.size() * sizeof(int4), hipMemcpyHostToDevice));
        CK(hipMalloc(&s->d_blocktab_ext, bte.size() * sizeof(int4)));
        CK(hipMemcpy(s->d_blocktab_ext, bte.data(), bte.size() * sizeof(int4), hipMemcpyHostToDevice));
        s->nblk_ext = (int)bte.size();
        CK(hipMalloc(&s->d_partial, bt.size() * sizeof(double)));
        CK(hipMemset(s->d_partial, 0, bt.size() * sizeof(double)));
    }
    s->have_mat = true;
    s->have_u = false;
    return MPX_OK;
}

mpx_status mpx_set_bias(mpx_sim *s, double hx, double hy, double hz) {
    mpx_status r = check_live(s);
    if (r != MPX_OK) return r;
    if (!std::isfinite(hx) || !std::isfinite(hy) || !std::isfinite(hz)) return fail(s, MPX_E_INVALID, "bias");
    s->H0[0] = hx;
    s->H0[1] = hy;
    s->H0[2] = hz;
    drop_graph(s);
    return MPX_OK;
}

mpx_status mpx_init_magnetization(mpx_sim *s, double ux, double uy, double uz) {
    mpx_status r = check_live(s);
    if (r != MPX_OK) return r;
    if (!s->have_mat) return fail(s, MPX_E_STATE, "init_magnetization before set_materials");
    const double nrm = std::sqrt(ux * ux + uy * uy + uz * uz);
    if (!(nrm > 0) || !std::isfinite(nrm)) return fail(s, MPX_E_INVALID, "direction");
    s->u[0] = ux / nrm;
    s->u[1] = uy / nrm;
    s->u[2] = uz / nrm;
    s->have_u = true;
    CK(hipStreamSynchronize(s->stream));
    for (auto &f : s->films) {
        std::vector<double> m(9 * f.ns, 0.0);
        for (int c = 0; c < 3; c++)
            for (long long l = 0; l < f.ns; l++) {
                const int idx[3] = {f.b0[0] + (int)(l % f.bn[0]), f.b0[1] + (int)((l / f.bn[0]) % f.bn[1]),
                                    f.b0[2] + (int)(l / ((long long)f.bn[0] * f.bn[1]))};
                double ms, al, ga;
                site_params_h(s, c, idx, ms, al, ga);
                for (int w = 0; w < 3; w++) m[(c * 3 + w) * f.ns + l] = ms > 0 ? ms * s->u[w] : 0.0;
            }
        CK(hipMemcpy(f.M, m.data(), m.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    return MPX_OK;
}

mpx_status mpx_add_source(mpx_sim *s, const mpx_source_desc *src, int32_t *id) {
    mpx_status r = check_live(s);
    if (r != MPX_OK) return r;
    if (!src || src->component < 0 || src->component > 2 || src->n_table < 0 || (!src->table && src->n_table > 0))
        return fail(s, MPX_E_INVALID, "bad source");
    if (src->ni < 0 || src->nj < 0 || src->nk < 0) return fail(s, MPX_E_INVALID, "bad source box");
    if ((int)s->srcs.size() >= kMaxSources) return fail(s, MPX_E_INVALID, "too many sources");
    SrcHost h{};
    h.dev.comp = src->component;
    const int b[6] = {src->i0, src->j0, src->k0, src->ni, src->nj, src->nk};
    for (int a = 0; a < 6; a++) h.dev.box[a] = b[a];
    h.dev.n = src->n_table;
    CK(hipMalloc(&h.table, std::max<int64_t>(1, src->n_table) * sizeof(double)));
    if (src->n_table > 0)
        CK(hipMemcpy(h.table, src->table, src->n_table * sizeof(double), hipMemcpyHostToDevice));
    h.dev.table = h.table;
    s->srcs.push_back(h);
    {
        std::vector<SrcDev> v;
        for (auto &x : s->srcs) v.push_back(x.dev);
        (void)hipFree(s->d_srcs);
        s->d_srcs = nullptr;
        CK(hipMalloc(&s->d_srcs, v.size() * sizeof(SrcDev)));
        CK(hipMemcpy(s->d_srcs, v.data(), v.size() * sizeof(SrcDev), hipMemcpyHostToDevice));
    }
    if ((r = update_pass_flags(s)) != MPX_OK) return r;
    drop_graph(s);
    if (id) *id = (int32_t)s->srcs.size() - 1;
    return MPX_OK;
}

mpx_status mpx_add_probe(mpx_sim *s, const mpx_probe_desc *pd, int32_t *id) {
    mpx_status r = check_live(s);
    if (r != MPX_OK) return r;
    if (!pd || pd->capacity < 1 || pd->kind < 0 || pd->kind > 3 || pd->every < 0)
        return fail(s, MPX_E_INVALID, "bad probe");
    if ((int)s->probes.size() >= kMaxProbes) return fail(s, MPX_E_INVALID, "too many probes");
    ProbeHost h{};
    h.dev.kind = pd->kind;
    h.dev.field = pd->field;
    h.dev.i = pd->i;
    h.dev.j = pd->j;
    h.dev.k = pd->k;
    h.dev.film = pd->film;
    h.dev.nval = pd->kind == MPX_PROBE_MEAN_M ? 3 : 1;
    h.dev.cap = pd->capacity;
    h.dev.start = s->step;
    h.dev.every = std::max(1, (int)pd->every);
    if (pd->kind == MPX_PROBE_FIELD) {
        if (pd->field < 0 || pd->field > 5) return fail(s, MPX_E_INVALID, "probe field");
        const int idx[3] = {pd->i, pd->j, pd->k};
        for (int a = 0; a < 3; a++)
            if (idx[a] < 0 || idx[a] >= natural_dim(s, pd->field, a)) return fail(s, MPX_E_INVALID, "probe index");
        if (pd->field >= 3) {
            const int c = pd->field - 3;
            for (int a = 0; a < 3; a++)
                if (a != c && idx[a] < s->n[a] && in_pml_cell(s, a, idx[a]))
                    return fail(s, MPX_E_UNSUPPORTED, "H probe inside a PML slab");
        }
    } else if (pd->kind == MPX_PROBE_EM_ENERGY) {
        if (!s->have_mat) return fail(s, MPX_E_STATE, "energy probe before set_materials");
        if (s->any_pml) return fail(s, MPX_E_UNSUPPORTED, "energy probe with PML faces");
    } else {
        if (!s->have_mat) return fail(s, MPX_E_STATE, "film probe before set_materials");
        if (pd->film < 0 || pd->film >= (int)s->films.size()) return fail(s, MPX_E_INVALID, "probe film");
    }
    CK(hipMalloc(&h.dev.data, pd->capacity * h.dev.nval * sizeof(double)));
    CK(hipMemset(h.dev.data, 0, pd->capacity * h.dev.nval * sizeof(double)));
    if (pd->kind == MPX_PROBE_FILM_ENERGY) {
        const int *cb = s->films[pd->film].cb;
        h.dev.npart = ((long long)cb[3] * cb[4] * cb[5] + 255) / 256;
        CK(hipMalloc(&h.dev.part, h.dev.npart * sizeof(double)));
    } else if (pd->kind == MPX_PROBE_EM_ENERGY) {
        h.dev.npart = ((long long)s->n[0] * s->n[1] * s->n[2] + 255) / 256;
        CK(hipMalloc(&h.dev.part, 2 * h.dev.npart * sizeof(double)));
    }
    s->probes.push_back(h);
    drop_graph(s);
    if ((r = upload_probes(s)) != MPX_OK) return r;
    if (id) *id = (int32_t)s->probes.size() - 1;
    return MPX_OK;
}

mpx_status mpx_step(mpx_sim *s, int64_t nsteps) {
    mpx_status r = check_live(s);
    if (r != MPX_OK) return r;
    if (nsteps < 0) return fail(s, MPX_E_INVALID, "negative step count");
    if (!s->have_mat) return fail(s, MPX_E_STATE, "step before set_materials");
    if (!s->films.empty() && !s->have_u) return fail(s, MPX_E_STATE, "step before init_magnetization");
    if (nsteps == 0) return MPX_OK;
    r = s->prec == MPX_F64 ? enqueue_steps<double>(s, nsteps) : enqueue_steps<float>(s, nsteps);
    if (r != MPX_OK) return r;
    s->step += nsteps;
    return MPX_OK;
}

mpx_status mpx_synchronize(mpx_sim *s) {
    mpx_status r = check_live(s);
    if (r != MPX_OK) return r;
    CK(hipStreamSynchronize(s->stream));
    int flag = 0;
    CK(hipMemcpy(&flag, s->d_flag, sizeof(int), hipMemcpyDeviceToHost));
    if (flag) return fail(s, MPX_E_NONFINITE, "a probe recorded a non-finite value");
    return MPX_OK;
}

// the stored values of a box (x0, y0, z0, nx, ny, nz) of an E or H slot
// array, clipped to the stored lattice, into a dense destination of that box
// (x fastest; zero where nothing is stored): one strided copy per plane on
// the handle's stream, device to device or device to host; synchronous
static mpx_status copy_box_out(mpx_sim *s, const void *src, const int64_t b[6], void *dst, bool dst_dev) {
    const size_t esz = s->esz;
    const size_t need = (size_t)(b[3] * b[4] * b[5]) * esz;
    if (dst_dev)
        CK(hipMemsetAsync(dst, 0, need, s->stream));
    else
        memset(dst, 0, need);
    const int64_t ci = std::min<int64_t>(b[3], s->n[0] - b[0]), cj = std::min<int64_t>(b[4], s->n[1] - b[1]);
    if (ci > 0 && cj > 0)
        for (int64_t k = 0; k < b[5]; k++) {
            const int64_t gk = b[2] + k;
            if (gk >= s->n[2]) break;
            const char *from = (const char *)src + (size_t)(b[0] + (int64_t)s->px * (b[1] + (int64_t)s->n[1] * gk)) * esz;
            char *to = (char *)dst + (size_t)(b[3] * b[4] * k) * esz;
            CK(hipMemcpy2DAsync(to, (size_t)b[3] * esz, from, (size_t)s->px * esz, (size_t)ci * esz, (size_t)cj,
                                dst_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s->stream));
        }
    CK(hipStreamSynchronize(s->stream));
    return MPX_OK;
}

mpx_status mpx_read_field(mpx_sim *s, int32_t field, void *dst, int64_t dst_bytes, int32_t dst_is_device) {
    mpx_status r = check_live(s);
    if (r != MPX_OK) return r;
    int64_t dims[4], bytes;
    if (field < 0 || field > 11 || !dst) return fail(s, MPX_E_INVALID, "bad field");
    mpx_query_field(s, field, dims, &bytes);
    if (dst_bytes < bytes) return fail(s, MPX_E_RANGE, "destination too small");
    CK(hipStreamSynchronize(s->stream));
    if (field < 6 && dst_is_device) {
        const int64_t b[6] = {0, 0, 0, dims[0], dims[1], dims[2]};
        return copy_box_out(s, field < 3 ? Eset(s, s->parity)[field] : Hset(s, s->parity)[field - 3], b, dst, true);
    }
    std::vector<char> host(bytes, 0);
    if (field < 6) {
        std::vector<char> slots(s->nslot * s->esz);
        void *src = field < 3 ? Eset(s, s->parity)[field] : Hset(s, s->parity)[field - 3];
        CK(hipMemcpy(slots.data(), src, slots.size(), hipMemcpyDeviceToHost));
        for (int64_t k = 0; k < dims[2]; k++)
            for (int64_t j = 0; j < dims[1]; j++) {
                if (k >= s->n[2] || j >= s->n[1]) continue;
                const int64_t ni = std::min<int64_t>(dims[0], s->n[0]);
                memcpy(&host[(size_t)(dims[0] * (j + dims[1] * k)) * s->esz],
                       &slots[(size_t)(s->px * (j + (int64_t)s->n[1] * k)) * s->esz], ni * s->esz);
            }
    } else {
        const int c = (field - 6) % 3;
        const bool delta = field >= 9;
        double *h = (double *)host.data();
        const int64_t nsite = dims[0] * dims[1] * dims[2];
        for (auto &f : s->films) {
            std::vector<double> m(9 * f.ns);
            CK(hipMemcpy(m.data(), f.M, m.size() * sizeof(double), hipMemcpyDeviceToHost));
            for (long long l = 0; l < f.ns; l++) {
                const int idx[3] = {f.b0[0] + (int)(l % f.bn[0]), f.b0[1] + (int)((l / f.bn[0]) % f.bn[1]),
                                    f.b0[2] + (int)(l / ((long long)f.bn[0] * f.bn[1]))};
                double ms, al, ga;
                site_params_h(s, c, idx, ms, al, ga);
                if (!(ms > 0)) continue;
                const int64_t q = idx[0] + dims[0] * (idx[1] + dims[1] * (int64_t)idx[2]);
                for (int w = 0; w < 3; w++) {
                    double v = m[(c * 3 + w) * f.ns + l];
                    if (delta) v -= (s->have_u ? ms * s->u[w] : 0.0);
                    h[w * nsite + q] = v;
                }
            }
        }
    }
    if (dst_is_device)
        CK(hipMemcpy(dst, host.data(), bytes, hipMemcpyHostToDevice));
    else
        memcpy(dst, host.data(), bytes);
    return MPX_OK;
}

mpx_status mpx_field_storage(mpx_sim *s, int32_t field, void **device_ptr, int64_t strides[3], int64_t *bytes) {
    mpx_status r = check_live(s);
    if (r != MPX_OK) return r;
    if (field < 0 || field > 5 || !device_ptr || !strides) return fail(s, MPX_E_INVALID, "bad field");
    if (s->fused) return fail(s, MPX_E_STATE, "the fused schedules move the fields between two buffers");
    *device_ptr = field < 3 ? Eset(s, s->parity)[field] : Hset(s, s->parity)[field - 3];
    strides[0] = 1;
    strides[1] = s->px;
    strides[2] = (int64_t)s->px * s->n[1];
    if (bytes) *bytes = s->nslot * (int64_t)s->esz;
    return MPX_OK;
}

mpx_status mpx_read_field_region(mpx_sim *s, int32_t field, const int32_t box[6], void *dst, int64_t dst_bytes,
                                 int32_t dst_is_device) {
    mpx_status r = check_live(s);
    if (r != MPX_OK) return r;
    int64_t dims[4], bytes;
    if (field < 0 || field > 11 || !dst || !box) return fail(s, MPX_E_INVALID, "bad field");
    mpx_query_field(s, field, dims, &bytes);
    for (int a = 0; a < 3; a++)
        if (box[a] < 0 || box[3 + a] < 0 || box[a] + box[3 + a] > dims[a]) return fail(s, MPX_E_INVALID, "bad box");
    const int64_t nr = (int64_t)box[3] * box[4] * box[5];
    const size_t esz = field < 6 ? s->esz : 8;
    const int64_t need = nr * dims[3] * (int64_t)esz;
    if (dst_bytes < need) return fail(s, MPX_E_RANGE, "destination too small");
    CK(hipStreamSynchronize(s->stream));
    if (field < 6) {
        if (nr == 0) return MPX_OK;
        const int64_t b[6] = {box[0], box[1], box[2], box[3], box[4], box[5]};
        return copy_box_out(s, field < 3 ? Eset(s, s->parity)[field] : Hset(s, s->parity)[field - 3], b, dst,
                            dst_is_device != 0);
    }
    std::vector<char> host(need, 0);
    {
        const int c = (field - 6) % 3;
        const bool delta = field >= 9;
        double *h = (double *)host.data();
        for (auto &f : s->films) {
            // intersect the film's face box with the region
            int lo[3], hi[3];
            bool empty = false;
            for (int a = 0; a < 3; a++) {
                lo[a] = std::max(f.b0[a], box[a]);
                hi[a] = std::min(f.b0[a] + f.bn[a], box[a] + box[3 + a]);
                if (hi[a] <= lo[a]) empty = true;
            }
            if (empty) continue;
            std::vector<double> m(9 * f.ns);
            CK(hipMemcpy(m.data(), f.M, m.size() * sizeof(double), hipMemcpyDeviceToHost));
            for (int k = lo[2]; k < hi[2]; k++)
                for (int j = lo[1]; j < hi[1]; j++)
                    for (int i = lo[0]; i < hi[0]; i++) {
                        const int idx[3] = {i, j, k};
                        double ms, al, ga;
                        site_params_h(s, c, idx, ms, al, ga);
                        if (!(ms > 0)) continue;
                        const long long l = (i - f.b0[0]) + (long long)f.bn[0] * ((j - f.b0[1]) + (long long)f.bn[1] * (k - f.b0[2]));
                        const int64_t q = (i - box[0]) + (int64_t)box[3] * ((j - box[1]) + (int64_t)box[4] * (k - box[2]));
                        for (int w = 0; w < 3; w++) {
                            double v = m[(c * 3 + w) * f.ns + l];
                            if (delta) v -= (s->have_u ? ms * s->u[w] : 0.0);
                            h[w * nr + q] = v;
                        }
                    }
        }
    }
    if (dst_is_device)
        CK(hipMemcpy(dst, host.data(), need, hipMemcpyHostToDevice));
    else
        memcpy(dst, host.data(), need);
    return MPX_OK;
}

mpx_status mpx_write_field(mpx_sim *s, int32_t field, const void *src, int64_t src_bytes, int32_t src_is_device) {
    mpx_status r = check_live(s);
    if (r != MPX_OK) return r;
    int64_t dims[4], bytes;
    if (field < 0 || field > 8 || !src) return fail(s, MPX_E_INVALID, "bad field");
    if (!s->have_mat) return fail(s, MPX_E_STATE, "write_field before set_materials");
    mpx_query_field(s, field, dims, &bytes);
    if (src_bytes < bytes) return fail(s, MPX_E_RANGE, "source too small");
    CK(hipStreamSynchronize(s->stream));
    std::vector<char> host(bytes);
    if (src_is_device)
        CK(hipMemcpy(host.data(), src, bytes, hipMemcpyDeviceToHost));
    else
        memcpy(host.data(), src, bytes);
    if (field < 6) {
        std::vector<char> slots(s->nslot * s->esz, 0);
        for (int64_t k = 0; k < std::min<int64_t>(dims[2], s->n[2]); k++)
            for (int64_t j = 0; j < std::min<int64_t>(dims[1], s->n[1]); j++)
                for (int64_t i = 0; i < std::min<int64_t>(dims[0], s->n[0]); i++) {
                    const int idx[3] = {(int)i, (int)j, (int)k};
                    if (field < 3 && edge_is_pec_h(s, field, idx)) continue;
                    memcpy(&slots[(size_t)(i + s->px * (j + (int64_t)s->n[1] * k)) * s->esz],
                           &host[(size_t)(i + dims[0] * (j + dims[1] * k)) * s->esz], s->esz);
                }
        void *dstp = field < 3 ? Eset(s, s->parity)[field] : Hset(s, s->parity)[field - 3];
        CK(hipMemcpy(dstp, slots.data(), slots.size(), hipMemcpyHostToDevice));
    } else {
        const int c = field - 6;
        const double *h = (const double *)host.data();
        const int64_t nsite = dims[0] * dims[1] * dims[2];
        for (auto &f : s->films) {
            std::vector<double> m(9 * f.ns);
            CK(hipMemcpy(m.data(), f.M, m.size() * sizeof(double), hipMemcpyDeviceToHost));
            for (long long l = 0; l < f.ns; l++) {
                const int idx[3] = {f.b0[0] + (int)(l % f.bn[0]), f.b0[1] + (int)((l / f.bn[0]) % f.bn[1]),
                                    f.b0[2] + (int)(l / ((long long)f.bn[0] * f.bn[1]))};
                double ms, al, ga;
                site_params_h(s, c, idx, ms, al, ga);
                if (!(ms > 0)) continue;
                const int64_t q = idx[0] + dims[0] * (idx[1] + dims[1] * (int64_t)idx[2]);
                for (int w = 0; w < 3; w++) m[(c * 3 + w) * f.ns + l] = h[w * nsite + q];
            }
            CK(hipMemcpy(f.M, m.data(), m.size() * sizeof(double), hipMemcpyHostToDevice));
        }
    }
    return MPX_OK;
}

mpx_status mpx_read_probe(mpx_sim *s, int32_t id, double *dst, int64_t capacity, int64_t *n_written) {
    mpx_status r = check_live(s);
    if (r != MPX_OK) return r;
    if (id < 0 || id >= (int)s->probes.size() || !n_written) return fail(s, MPX_E_INVALID, "bad probe id");
    const ProbeDev &P = s->probes[id].dev;
    const long long samples = (s->step - P.start) / std::max(1, P.every);
    const long long have = std::min<long long>(samples, P.cap);
    *n_written = have;
    if (capacity < have || (!dst && have > 0)) return fail(s, MPX_E_RANGE, "probe destination too small");
    CK(hipStreamSynchronize(s->stream));
    std::vector<double> buf(P.cap * P.nval);
    CK(hipMemcpy(buf.data(), P.data, buf.size() * sizeof(double), hipMemcpyDeviceToHost));
    const long long first = samples - have;
    for (long long t = 0; t < have; t++) {
        const long long slot = (first + t) % P.cap;
        for (int w = 0; w < P.nval; w++) dst[t * P.nval + w] = buf[slot * P.nval + w];
    }
    return MPX_OK;
}

mpx_status mpx_energy(mpx_sim *s, double *W_em, double *W_z) {
    mpx_status r = check_live(s);
    if (r != MPX_OK) return r;
    if (!W_em || !W_z) return MPX_E_INVALID;
    if (!s->have_mat) return fail(s, MPX_E_STATE, "energy before set_materials");
    if (s->any_pml) return fail(s, MPX_E_UNSUPPORTED, "energy with PML faces");
    const long long nb = (long long)((s->n[0] + 63) / 64) * ((s->n[1] + 3) / 4) * s->n[2];
    double *part = nullptr, *out = nullptr;
    CK(hipMalloc(&part, 2 * nb * sizeof(double)));
    CK(hipMalloc(&out, 3 * sizeof(double)));
    CK(hipMemsetAsync(out, 0, 3 * sizeof(double), s->stream));
    hipError_t e;
    if (s->prec == MPX_F64) {
        KParams<double> p;
        fill_params<double>(s, p);
        e = launch_energy<double>(p, s->nblk, part, out, s->stream);
    } else {
        KParams<float> p;
        fill_params<float>(s, p);
        e = launch_energy<float>(p, s->nblk, part, out, s->stream);
    }
    if (e != hipSuccess) return dev_fail(s, e, "energy kernels");
    double h[3];
    CK(hipStreamSynchronize(s->stream));
    CK(hipMemcpy(h, out, sizeof(h), hipMemcpyDeviceToHost));
    (void)hipFree(part);
    (void)hipFree(out);
    const double dV = s->d[0] * s->d[1] * s->d[2];
    *W_em = 0.5 * dV * (h[0] + MU0 * h[1]);
    *W_z = -MU0 * dV * h[2];
    return MPX_OK;
}

mpx_status mpx_energy_noalloc(mpx_sim *s, double *W_em, double *W_z) {
    mpx_status r = check_live(s);
    if (r != MPX_OK) return r;
    if (!W_em || !W_z) return MPX_E_INVALID;
    if (!s->have_mat) return fail(s, MPX_E_STATE, "energy before set_materials");
    if (s->any_pml) return fail(s, MPX_E_UNSUPPORTED, "energy with PML faces");
    const long long nb = (long long)((s->n[0] + 63) / 64) * ((s->n[1] + 3) / 4) * s->n[2];
    if (kScratchPart + 2 * nb > kScratchDoubles)
        return fail(s, MPX_E_RANGE, "grid too large for the no-allocation energy (at most 1048560 blocks of 64 x 4 cells)");
    double *scr = nullptr;
    if ((r = energy_scratch_ptr(s, &scr)) != MPX_OK) return r;
    double *out = scr, *part = scr + kScratchPart;
    hipLaunchKernelGGL(k_clear3, dim3(1), dim3(64), 0, s->stream, out);
    hipError_t e;
    if (s->prec == MPX_F64) {
        KParams<double> p;
        fill_params<double>(s, p);
        e = launch_energy<double>(p, s->nblk, part, out, s->stream);
    } else {
        KParams<float> p;
        fill_params<float>(s, p);
        e = launch_energy<float>(p, s->nblk, part, out, s->stream);
    }
    if (e != hipSuccess) return dev_fail(s, e, "energy kernels");
    double h[3];
    CK(hipStreamSynchronize(s->stream));
    CK(hipMemcpy(h, out, sizeof(h), hipMemcpyDeviceToHost));
    const double dV = s->d[0] * s->d[1] * s->d[2];
    *W_em = 0.5 * dV * (h[0] + MU0 * h[1]);
    *W_z = -MU0 * dV * h[2];
    return MPX_OK;
}

mpx_status mpx_info(const mpx_sim *s, int64_t *step, double *time, double *dt, int32_t *n_films) {
    if (!s) return MPX_E_INVALID;
    if (step) *step = s->step;
    if (time) *time = s->step * s->dt;
    if (dt) *dt = s->dt;
    if (n_films) *n_films = (int32_t)s->films.size();
    return MPX_OK;
}

mpx_status mpx_film_box(const mpx_sim *s, int32_t film, int32_t box[6], int64_t *ncells) {
    if (!s || !box || film < 0 || film >= (int)s->films.size()) return MPX_E_INVALID;
    for (int a = 0; a < 6; a++) box[a] = s->films[film].cb[a];
    if (ncells) *ncells = s->films[film].ncells;
    return MPX_OK;
}

mpx_status mpx_set_graph_steps(mpx_sim *s, int32_t steps) {
    if (!s || steps < 0) return MPX_E_INVALID;
    if (steps != s->graph_steps) drop_graph(s);
    s->graph_steps = steps;
    return MPX_OK;
}

mpx_status mpx_set_timing(mpx_sim *s, int32_t every) {
    if (!s || every < 0) return MPX_E_INVALID;
    if (every != s->timing_every) drop_graph(s); // the untimed runs' graphs have its length
    s->timing_every = every;
    return MPX_OK;
}

mpx_status mpx_kernel_time(mpx_sim *s, double *avg_ms, int64_t *launches) {
    if (!s || !avg_ms || !launches) return MPX_E_INVALID;
    for (int g = 0; g < 3; g++) {
        avg_ms[g] = s->t_n[g] ? s->t_ms[g] / s->t_n[g] : 0.0;
        launches[g] = s->t_n[g];
    }
    return MPX_OK;
}

mpx_status mpx_set_schedule(mpx_sim *s, int32_t fused, int32_t kchunk) {
    if (!s || kchunk < 0) return MPX_E_INVALID;
    if (fused < 0 || fused > 6) return MPX_E_INVALID;
    drop_graph(s);
    s->narrow = fused == 6;
    s->fused = fused == 6 ? 0 : fused;
    if (kchunk > 0) s->kchunk = kchunk;
    return MPX_OK;
}

const char *mpx_last_error(const mpx_sim *s) { return s ? s->err.c_str() : "null handle"; }

mpx_status mpx_adjoint(mpx_sim *s, int64_t nsteps, int64_t loss_from, int32_t film, int32_t checkpoint_every,
                       const int32_t eps_box[6], const int32_t ms_box[6], double *loss, double *dL_dH0,
                       double *dL_deps, double *dL_dMs) {
    mpx_status r = check_live(s);
    if (r != MPX_OK) return r;
    if (!s->have_mat) return fail(s, MPX_E_STATE, "adjoint before set_materials");
    if (!s->films.empty() && !s->have_u) return fail(s, MPX_E_STATE, "adjoint before init_magnetization");
    if (nsteps < 1 || loss_from < 0 || loss_from >= nsteps || film < 0 || film >= (int)s->films.size() ||
        checkpoint_every < 0 || !eps_box || !ms_box || !loss || !dL_dH0)
        return fail(s, MPX_E_INVALID, "adjoint arguments");
    for (int a = 0; a < 3; a++)
        if (eps_box[3 + a] < 0 || ms_box[3 + a] < 0 || eps_box[a] < 0 || ms_box[a] < 0 ||
            eps_box[a] + eps_box[3 + a] > s->n[a] || ms_box[a] + ms_box[3 + a] > s->n[a])
            return fail(s, MPX_E_INVALID, "adjoint box outside the grid");
    if ((long long)eps_box[3] * eps_box[4] * eps_box[5] > 0 && !dL_deps) return fail(s, MPX_E_INVALID, "dL_deps");
    if ((long long)ms_box[3] * ms_box[4] * ms_box[5] > 0 && !dL_dMs) return fail(s, MPX_E_INVALID, "dL_dMs");
    int K = checkpoint_every;
    if (K == 0) K = std::max(1, (int)std::ceil(std::sqrt((double)nsteps)));
    K = (int)std::min<int64_t>(K, nsteps);
    drop_graph(s);
    AdjLoss ls;
    ls.film = film;
    ls.loss_from = loss_from;
    if (s->adj_schedule != 1)
        r = s->prec == MPX_F64 ? run_adjoint_tape<double>(s, nsteps, ls, K, eps_box, ms_box, loss, dL_dH0, dL_deps, dL_dMs)
                               : run_adjoint_tape<float>(s, nsteps, ls, K, eps_box, ms_box, loss, dL_dH0, dL_deps, dL_dMs);
    else
        r = s->prec == MPX_F64
                ? run_adjoint<double>(s, nsteps, loss_from, film, K, eps_box, ms_box, loss, dL_dH0, dL_deps, dL_dMs)
                : run_adjoint<float>(s, nsteps, loss_from, film, K, eps_box, ms_box, loss, dL_dH0, dL_deps, dL_dMs);
    return r;
}

mpx_status mpx_adjoint_probe(mpx_sim *s, int64_t nsteps, int32_t field, const int32_t ijk[3], const double *weights,
                             int32_t checkpoint_every, const int32_t eps_box[6], const int32_t ms_box[6], double *loss,
                             double *dL_dH0, double *dL_deps, double *dL_dMs) {
    mpx_status r = check_live(s);
    if (r != MPX_OK) return r;
    if (!s->have_mat) return fail(s, MPX_E_STATE, "adjoint before set_materials");
    if (!s->films.empty() && !s->have_u) return fail(s, MPX_E_STATE, "adjoint before init_magnetization");
    if (s->adj_schedule == 1) return fail(s, MPX_E_UNSUPPORTED, "a weighted-trace loss needs the tape schedule");
    if (nsteps < 1 || field < 0 || field > 2 || !ijk || !weights || checkpoint_every < 0 || !eps_box || !ms_box ||
        !loss || !dL_dH0)
        return fail(s, MPX_E_INVALID, "adjoint arguments");
    for (int a = 0; a < 3; a++)
        if (ijk[a] < 0 || ijk[a] >= s->n[a]) return fail(s, MPX_E_INVALID, "probe edge outside the stored sites");
    for (int a = 0; a < 3; a++)
        if (eps_box[3 + a] < 0 || ms_box[3 + a] < 0 || eps_box[a] < 0 || ms_box[a] < 0 ||
            eps_box[a] + eps_box[3 + a] > s->n[a] || ms_box[a] + ms_box[3 + a] > s->n[a])
            return fail(s, MPX_E_INVALID, "adjoint box outside the grid");
    if ((long long)eps_box[3] * eps_box[4] * eps_box[5] > 0 && !dL_deps) return fail(s, MPX_E_INVALID, "dL_deps");
    if ((long long)ms_box[3] * ms_box[4] * ms_box[5] > 0 && !dL_dMs) return fail(s, MPX_E_INVALID, "dL_dMs");
    for (int64_t i = 0; i < nsteps; i++)
        if (!std::isfinite(weights[i])) return fail(s, MPX_E_INVALID, "weights must be finite");
    int K = checkpoint_every;
    if (K == 0) K = std::max(1, (int)std::ceil(std::sqrt((double)nsteps)));
    K = (int)std::min<int64_t>(K, nsteps);
    drop_graph(s);
    AdjLoss ls;
    ls.kind = 1;
    ls.field = field;
    for (int a = 0; a < 3; a++) ls.ijk[a] = ijk[a];
    ls.w = weights;
    return s->prec == MPX_F64
               ? run_adjoint_tape<double>(s, nsteps, ls, K, eps_box, ms_box, loss, dL_dH0, dL_deps, dL_dMs)
               : run_adjoint_tape<float>(s, nsteps, ls, K, eps_box, ms_box, loss, dL_dH0, dL_deps, dL_dMs);
}

mpx_status mpx_set_adjoint_schedule(mpx_sim *s, int32_t schedule) {
    mpx_status r = check_live(s);
    if (r != MPX_OK) return r;
    if (schedule < 0 || schedule > 2) return fail(s, MPX_E_INVALID, "adjoint schedule");
    s->adj_schedule = schedule;
    return MPX_OK;
}

mpx_status mpx_set_adjoint_memory(mpx_sim *s, int64_t max_bytes) {
    mpx_status r = check_live(s);
    if (r != MPX_OK) return r;
    if (max_bytes < -1) return fail(s, MPX_E_INVALID, "adjoint memory");
    s->adj_resident = max_bytes;
    return MPX_OK;
}


mpx_status mpx_batch_create(mpx_sim *const *sims, int32_t n, mpx_batch **out) {
    if (!sims || n < 1 || !out) return MPX_E_INVALID;
    *out = nullptr;
    for (int q = 0; q < n; q++) {
        if (!sims[q] || sims[q]->dead) return MPX_E_INVALID;
        if (!sims[q]->have_mat || (!sims[q]->films.empty() && !sims[q]->have_u)) return MPX_E_STATE;
        if (sims[q]->prec != sims[0]->prec || sims[q]->device != sims[0]->device) return MPX_E_INVALID;
        for (int r = 0; r < q; r++)
            if (sims[r] == sims[q]) return MPX_E_INVALID;
    }
    mpx_batch *b = new mpx_batch();
    b->sims.assign(sims, sims + n);
    b->prec = sims[0]->prec;
    b->device = sims[0]->device;
    b->stream = sims[0]->stream;
    b->variant = sims[0]->fused;
    b->kchunk = sims[0]->kchunk;
    (void)hipSetDevice(b->device);
    b->psize = b->prec == MPX_F64 ? sizeof(KParams<double>) : sizeof(KParams<float>);
    mpx_status r = MPX_OK;
    auto setup = [&]() -> mpx_status {
        for (int f = 0; f < 2; f++) {
            BCK(hipMalloc(&b->d_pa[f], n * b->psize));
            BCK(hipMalloc(&b->d_pb[f], n * b->psize));
        }
        return b->prec == MPX_F64 ? batch_tables<double>(b) : batch_tables<float>(b);
    };
    r = setup();
    if (r != MPX_OK) {
        mpx_batch_destroy(b);
        return r;
    }
    *out = b;
    return MPX_OK;
}

mpx_status mpx_batch_destroy(mpx_batch *b) {
    if (!b) return MPX_OK;
    (void)hipSetDevice(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    batch_drop_graph(b);
    for (auto e : b->ev) (void)hipEventDestroy(e);
    for (int f = 0; f < 2; f++) {
        (void)hipFree(b->d_pa[f]);
        (void)hipFree(b->d_pb[f]);
    }
    (void)hipFree(b->d_work);
    (void)hipFree(b->d_work2);
    (void)hipFree(b->d_wmixed);
    (void)hipFree(b->d_wfilm);
    (void)hipFree(b->d_wext);
    (void)hipFree(b->d_wprobe);
    (void)hipFree(b->d_tick);
    delete b;
    return MPX_OK;
}

mpx_status mpx_batch_set_schedule(mpx_batch *b, int32_t variant, int32_t kchunk) {
    if (!b || variant < 0 || variant > 5 || kchunk < 0) return MPX_E_INVALID;
    (void)hipSetDevice(b->device);
    batch_drop_graph(b);
    const bool retile = variant != b->variant || (kchunk > 0 && kchunk != b->kchunk);
    b->variant = variant;
    if (kchunk > 0) b->kchunk = kchunk;
    if (retile) return b->prec == MPX_F64 ? batch_tables<double>(b) : batch_tables<float>(b);
    return MPX_OK;
}

mpx_status mpx_batch_set_graph_steps(mpx_batch *b, int32_t steps) {
    if (!b || steps < 0) return MPX_E_INVALID;
    if (steps != b->graph_steps) batch_drop_graph(b);
    b->graph_steps = steps;
    return MPX_OK;
}

mpx_status mpx_batch_step(mpx_batch *b, int64_t nsteps) {
    if (!b || nsteps < 0) return MPX_E_INVALID;
    if (b->dead) return MPX_E_DEVICE;
    for (mpx_sim *s : b->sims)
        if (s->dead) return MPX_E_DEVICE;
    if (nsteps == 0) return MPX_OK;
    hipError_t e = hipSetDevice(b->device);
    if (e != hipSuccess) return bdev_fail(b, e, "hipSetDevice");
    // order the batch stream after each instance's own stream, and back
    auto join = [&](hipStream_t from, hipStream_t to) -> mpx_status {
        if (from == to) return MPX_OK;
        hipEvent_t ev;
        BCK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        BCK(hipEventRecord(ev, from));
        BCK(hipStreamWaitEvent(to, ev, 0));
        b->ev.push_back(ev);
        return MPX_OK;
    };
    mpx_status r;
    for (mpx_sim *s : b->sims)
        if ((r = join(s->stream, b->stream)) != MPX_OK) return r;
    r = b->prec == MPX_F64 ? batch_steps<double>(b, nsteps) : batch_steps<float>(b, nsteps);
    if (r != MPX_OK) return r;
    for (mpx_sim *s : b->sims)
        if ((r = join(b->stream, s->stream)) != MPX_OK) return r;
    if (b->ev.size() > 4096) {
        BCK(hipStreamSynchronize(b->stream));
        for (auto ev : b->ev) (void)hipEventDestroy(ev);
        b->ev.clear();
    }
    return MPX_OK;
}

mpx_status mpx_batch_synchronize(mpx_batch *b) {
    if (!b) return MPX_E_INVALID;
    if (b->dead) return MPX_E_DEVICE;
    BCK(hipStreamSynchronize(b->stream));
    for (mpx_sim *s : b->sims) {
        mpx_status r = mpx_synchronize(s);
        if (r != MPX_OK) return r;
    }
    return MPX_OK;
}

const char *mpx_batch_last_error(const mpx_batch *b) { return b ? b->err.c_str() : "null handle"; }


} // extern "C"
