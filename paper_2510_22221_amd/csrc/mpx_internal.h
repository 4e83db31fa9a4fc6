// mpx_internal.h -- device-side data structures of libmpx and the launcher
// declarations shared by kernels.hip and host.hip.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpx {

constexpr int kMaxSources = 16;
constexpr int kMaxProbes = 64;
constexpr int kMaxFilms = 64;

struct MatDev {
    double eps_r, sigma, Ms, alpha, gamma_abs;
    int is_pec, pad;
};

// A film: cell box cb (i0,j0,k0,ni,nj,nk), the slot box of its face sites
// (b0, bn; the cell box grown by one face on each non-spanned axis), and the
// magnetisation of every face family stored over that box, float64:
//   M [family][component][site], the state
//   M1[family][component][site], H1[family][site], the scratch of the first
//   half step of a merged pair (the values at the integer time)
struct FilmDev {
    int b0[3], bn[3];
    int cb[6];
    long long ns;
    double ncells;
    double *M, *M1, *H1;
    const double *prm; // [family][Ms_s, alpha_s, |gamma|_s][site], from the ids
    int blk0[3], nblk[3];
    // B^ and B^* of every face of the face box grown by one layer on the low
    // side of each axis it does not span (the neighbours the LLG reads),
    // [family][site], written by a prepass before each half step
    int e0[3], en[3];
    long long nse;
    double *Bn, *Bs;
    // the same for the next half step of a merged pair, written by the
    // kernels of the first (both half steps use one E, so the first knows
    // every input of the second's prepass): the second reads these and runs
    // no prepass of its own (null: not written)
    double *Bn2, *Bs2;
};

struct SrcDev {
    int comp;
    int box[6];
    long long n;
    const double *table;
};

struct ProbeDev {
    int kind, field, i, j, k, film, nval, every; // every <= 1: each step
    long long cap, start;
    double *data;
    double *part;    // film-energy probes: one partial sum per 256 cells of the film's cell box;
                     // EM-energy probes: two (E and H sums) per 256 cells of the grid
    long long npart;
};

// a probe the merged H/M launch can take (it reads nothing that launch
// writes): a point probe of an E component (kind 0, field below 3) or a
// film's mean M (kind 1)
__host__ __device__ inline bool probe_reads_e_or_m(int kind, int field) {
    return (kind == 0 && field < 3) || kind == 1;
}

// Coefficients of an edge, computed on the host with the same operation
// sequence the device uses for mixed edges (so the table path is bitwise
// identical to the general one).  The table holds kCoefPerClass entries per
// slot class, one per edge component: a class below the number of materials
// is that material (its three entries equal); a class from there up to 254 is
// a compound class, one distinct triple of edge coefficients of slots whose
// eight cells do not share one id; 255 (kMixed) has no entries.
template <typename T>
struct CoefDev {
    T ca, cb;
    int pec, pad;
};
constexpr int kMixed = 255; // class byte of a slot whose edges take the general path
constexpr int kCoefPerClass = 3;
constexpr int kCoefEntries = kCoefPerClass * 256;
// values per packed row (coefv): six, float rows padded to 32 bytes
template <typename T>
constexpr int kCoefRow = sizeof(T) == 4 ? 8 : 6;

template <typename T>
struct KParams {
    int n[3];
    int px;
    int per[3];
    double d[3];
    T dT[3];
    T invd[3];
    T hc;        // dt / (2 mu0)
    double hcd;  // the same in float64
    double dt, inv_dt, eps0, mu0, kf, dV;
    double H0[3];
    T *E[3];
    T *H[3];
    T *Hw[3];      // where the film kernels write H of magnetic faces
    T *Eb[3];      // fused pass: destinations (ping-pong partners of E, H)
    T *Hb[3];
    T *psiEb[3][3];
    const CoefDev<T> *coef;
    // every distinct edge-coefficient triple of the mixed-class slots (up to
    // 2^20 of them), three entries each: the same allocation as coef, after
    // its kCoefEntries class entries
    const CoefDev<T> *coefx;
    // the same rows packed for the separate E pass: row r (a class, or 256 +
    // an extended triple) holds ca, cb of its x, y and z edges side by side
    // (kCoefRow values; float rows padded to eight), so that one or two wide
    // loads fetch a slot's six coefficients
    const T *coefv;
    const uint8_t *id;
    const uint8_t *cls; // per slot: the shared id of the 8 cells around it, or 255
    const uint8_t *pflags; // per separate-pass tile: 1 CPML, 2 source, 4 film within reach
    // wide = 1: the single-instance passes use 256 x 1 tiles (rows of at least
    // two tiles), with their flags in pflags_w; batches keep the 64 x 4 tiles
    const uint8_t *pflags_w;
    int wide;
    // slots of the mixed class left out of the 16-bit classes: (i, j, k,
    // their extended-table index, or -1 for the general path from the cell
    // ids)
    const int4 *mixed;
    int nmixed;
    // per slot, when the extended table has entries (else null): the class
    // byte's value below 255, or 256 + the extended triple's index (rows of
    // coef after the 256 classes'), or 0xffff for a slot on the mixed list
    const uint16_t *cls16;
    const MatDev *mat;
    int nlo[3], nhi[3];
    const T *bE[3];
    const T *cE[3];
    const T *bH[3];
    const T *cH[3];
    T *psiE[3][3]; // [component][derivative axis]
    T *psiH[3][3];
    int nfilm;
    const FilmDev *films;
    const int4 *blocktab;
    const int4 *blocktab_ext; // blocks of the B^ prepass (film, family, first)
    int nblk_ext;
    double *partial;
    int nsrc;
    SrcDev src[kMaxSources];
    const SrcDev *srcs; // the same sources in device memory
    const ProbeDev *probes;
    long long *step;
    int *flag;

    __host__ __device__ long long slot(int i, int j, int k) const {
        return (long long)i + (long long)px * ((long long)j + (long long)n[1] * k);
    }
    // CPML slab storage along axis w: slab position sp in [0, nlo + nhi)
    __host__ __device__ long long psi_index(int w, const int *idx) const {
        const int S = nlo[w] + nhi[w];
        const int p = idx[w];
        const int sp = p < nlo[w] ? p : nlo[w] + (p - (n[w] - nhi[w]));
        if (w == 0) return (long long)sp + (long long)S * ((long long)idx[1] + (long long)n[1] * idx[2]);
        if (w == 1) return (long long)idx[0] + (long long)px * ((long long)sp + (long long)S * idx[2]);
        return (long long)idx[0] + (long long)px * ((long long)idx[1] + (long long)n[1] * sp);
    }
};

// one contiguous device-to-device copy of a snapshot table (bytes: a multiple
// of 4; both ends 16-byte aligned)
struct CopySeg {
    const void *src;
    void *dst;
    long long bytes;
};

// adjoint arrays of one film (layouts of FilmDev::M)
struct AdjFilmDev {
    double *lM;    // [family][component][site] lambda of M (in: after the map)
    double *lMout; // [family][component][site] lambda of M before the map
    double *lp;    // [family][component][site] lambda of P (own and transverse)
    double *lq;    // the same for Q
    double *gMs;   // [family][site] accumulated dL/dMs of the face
    double *gH0;   // [family][component][site] accumulated dL/dH0 parts
    // fused schedule: the film's reach (faces within one slot of its face
    // box; a whole periodic axis) and the curl-part adjoints of its faces,
    // [family][aD0 | aD1][region slot]
    double *aDr;
    long long nr;
    int r0[3], rn[3];
};

template <typename T>
struct AdjParams {
    KParams<T> p;          // the map's input state (E, H, psi, film M, prepass)
    T *lE[3], *lH[3];      // lambda of E and H (in place: after -> before)
    T *lpsiE[3][3], *lpsiH[3][3];
    T *aD[3][2];           // per face: lambda of the two curl parts of E
    T *eD[3][2];           // per edge: lambda of the two curl parts of H
    double *gca[3], *gcb[3]; // per edge: accumulated dL/dca, dL/dcb
    const AdjFilmDev *af;
    // the merged pass of two half-step transposes (the first half step of
    // step m, then the second of step m - 1): the film tables of the second
    const AdjFilmDev *afb;
    // fused schedule: destination set of lambda psiH (read from lpsiH), the
    // second lambda psiE set (the E-step adjoint of step n reads set n & 1
    // and writes the other), per-tile flags (1 CPML, 4 film reach, with a
    // two-slot halo), the segment's first step on the device, the step's
    // index in the segment
    T *lpsiHo[3][3];
    T *lpsiE2[3][3];
    T *mu[3];              // per edge: cb lambda E' (written by the second half-step pass)
    // folded into the first half-step pass: dL/dca, dL/dcb over the eps box
    // (btape: E^n and x^n of the box's edges; null for no box), and the loss
    // term of the state at the step's start (ltape: the film region's E and H)
    const double *btape;
    double *gca_box, *gcb_box;
    int bb[3], bs[3];
    const double *ltape;
    int lfilm;
    double lscale;
    long long loss_from;
    // a weighted-trace loss: weight pw[n - 1] of E component pw_comp at slot
    // pw_slot for the state at time n (pw null: none), scaled by pw_scale
    const double *pw = nullptr;
    long long pw_slot = -1;
    int pw_comp = 0;
    double pw_scale = 1.0;
    const uint8_t *aflags;
    const long long *seg0;
    int m;
};

template <typename T> hipError_t launch_adj_half(const AdjParams<T> &A, int nblk, hipStream_t s);
// tape schedule: the film-region and box-region tapes and their adjoint kernels
template <typename T>
hipError_t launch_tape_loss(const KParams<T> &p, int film, int merged, double *dst, hipStream_t s, const int *cb);
template <typename T>
hipError_t launch_adj_loss_tape(const AdjParams<T> &A, int film, double scale, const double *tape,
                                const long long *seg0, int m, long long loss_from, hipStream_t s, const int *cb);
template <typename T> hipError_t launch_tape_box(const KParams<T> &p, const int *box, double *dst, hipStream_t s);
template <typename T>
hipError_t launch_adj_eps_box(const KParams<T> &p, const int *box, const double *gca, const double *gcb, double *out,
                              hipStream_t s);
hipError_t launch_copy_segs(const CopySeg *segs, int nseg, int nblk, hipStream_t s);
template <typename T> hipError_t launch_add_one(T *a, long long q, double v, hipStream_t s);
// the film-energy loss's own eps_r term of the film cells, accumulated per
// cell of the film's cell box from a tape slot or from the current state
template <typename T>
hipError_t launch_adj_loss_eps_tape(const KParams<T> &p, int film, double scale, const double *tape,
                                    const long long *seg0, int m, long long loss_from, double *acc, hipStream_t s,
                                    const int *cb);
template <typename T>
hipError_t launch_adj_loss_eps_state(const KParams<T> &p, int film, double scale, double *acc, hipStream_t s,
                                     const int *cb);
long long film_tape_size(const int *cb);
long long box_tape_size(const int *box);
// fused schedule: the half-step adjoint (scale = 1: first apply the E step's
// lambda E = ca lambda E') and the E-step adjoint as one stencil pass each
template <typename T>
hipError_t launch_adj_half_fused(const AdjParams<T> &A, int nblk, int scale, const long long *film_nr, hipStream_t s);
template <typename T>
hipError_t launch_adj_film_part(const AdjParams<T> &A, int nblk, const long long *film_nr, hipStream_t s);
template <typename T> hipError_t launch_adj_hfield2(const AdjParams<T> &A, hipStream_t s);
template <typename T> hipError_t launch_adj_loss_h(const AdjParams<T> &A, const int *film_cb, hipStream_t s);
template <typename T> hipError_t launch_adj_estep_fused(const AdjParams<T> &A, hipStream_t s);
template <typename T> hipError_t launch_adj_estep(const AdjParams<T> &A, hipStream_t s);
template <typename T> hipError_t launch_adj_loss(const AdjParams<T> &A, int film, double scale, hipStream_t s);
template <typename T> hipError_t launch_adj_eps(const AdjParams<T> &A, const int *box, double *out, hipStream_t s);
template <typename T>
hipError_t launch_film_energy(const KParams<T> &p, int film, double *part, double *acc, double scale, hipStream_t s);
hipError_t launch_set_step(long long *step, long long v, hipStream_t s);
template <typename T> hipError_t launch_bhat(const KParams<T> &p, int phase, hipStream_t s);
hipError_t launch_adj_init_ms(const int4 *blocktab, int nblk, const FilmDev *films, const AdjFilmDev *af,
                              const double *u, hipStream_t s);
template <typename T> hipError_t launch_hbulk(const KParams<T> &p, int nhalf, int inc, hipStream_t s);
template <typename T> hipError_t launch_epass(const KParams<T> &p, hipStream_t s);
template <typename T>
hipError_t launch_epass_batch(const KParams<T> *plist, const int4 *work, int nwork, const int2 *mwork, int nmwork,
                              bool xcls, hipStream_t s);
template <typename T>
hipError_t launch_hbulk_batch(const KParams<T> *plist, const int4 *work, int nwork, int nhalf, int inc,
                              hipStream_t s);
int pass_tiles(const int *n);
constexpr int kPassTX = 64, kPassTY = 4; // separate-pass tile: 64 x 4 slots of one plane
constexpr int kWideTX = 256, kWideTY = 1; // the wide tile of the single-instance passes
constexpr int kWideMinNx = 512;           // grids this wide use it

// the bulk H/M pass with the film's second half step (and, nprobe > 0, the
// probes, all of kinds probe_reads_e_or_m accepts; 256 x 1 tiles and films only)
template <typename T>
hipError_t launch_hbulk_film(const KParams<T> &p, int nblk, int inc, hipStream_t s, int nprobe = 0);
template <typename T> hipError_t launch_film(const KParams<T> &p, int nblk, int phase, int inc, hipStream_t s);
template <typename T> hipError_t launch_fused(const KParams<T> &p, int kchunk, int variant, hipStream_t s);
template <typename T> hipError_t launch_sweep(const KParams<T> &p, int kchunk, hipStream_t s);
template <typename T>
hipError_t launch_sweep_batch(const KParams<T> *plist, const int4 *work, int nwork, hipStream_t s);
int sweep_tiles(const int *n, int kchunk);
hipError_t launch_classify(const uint8_t *id, uint8_t *cls, const int *n, const int *per, int px, hipStream_t s);
hipError_t launch_tick(long long *step, hipStream_t s);
template <typename T>
hipError_t launch_fused_batch(const KParams<T> *plist, const int4 *work, int nwork, int variant, hipStream_t s);
template <typename T>
hipError_t launch_film_batch(const KParams<T> *plist, const int2 *work_ext, int n_ext, const int2 *work, int n,
                             int phase, int inc, hipStream_t s);
template <typename T>
hipError_t launch_probes_batch(const KParams<T> *plist, const int2 *work, int n, int maxpart, hipStream_t s);
template <typename T> hipError_t launch_tick_batch(const KParams<T> *plist, const int *inst, int n, hipStream_t s);
template <typename T> hipError_t launch_commit(const KParams<T> &p, int nblk, hipStream_t s);
template <typename T> hipError_t launch_probes(const KParams<T> &p, int nprobe, int maxpart, hipStream_t s);
template <typename T>
hipError_t launch_energy(const KParams<T> &p, int nblk, double *part, double *out, hipStream_t s);

} // namespace mpx
