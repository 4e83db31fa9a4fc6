// device_common.h -- small device helpers shared by the kernel files.
#pragma once

#include "mpx_internal.h"

namespace mpx {

// index along an axis of extent n: wrapped once on a periodic axis; -1 when
// outside the domain (or still outside after one wrap)
__device__ __forceinline__ int fold(int i, int n, int per) {
    if (per) {
        if (i < 0)
            i += n;
        else if (i >= n)
            i -= n;
    }
    return (i < 0 || i >= n) ? -1 : i;
}

// central difference over a spacing: a true division in float64 (the plain
// definition), a multiply by the reciprocal in float32
template <typename T>
__device__ __forceinline__ T dif(T hi, T lo, T d, T invd) {
    if constexpr (sizeof(T) == 8) {
        (void)invd;
        return (hi - lo) / d;
    } else {
        (void)d;
        return (hi - lo) * invd;
    }
}

// value of a field at (i, j, k), folded on periodic axes; zero outside the
// domain (the walls' unstored sites)
template <typename T>
__device__ __forceinline__ T ldz(const KParams<T> &p, const T *a, int i, int j, int k) {
    int ii = fold(i, p.n[0], p.per[0]), jj = fold(j, p.n[1], p.per[1]), kk = fold(k, p.n[2], p.per[2]);
    if (ii < 0 || jj < 0 || kk < 0) return T(0);
    return a[p.slot(ii, jj, kk)];
}

// a film descriptor and a film-block table entry read through the scalar
// cache (both tables are uniform per block and read-only within a launch):
// their waits do not hold vector loads, and scalar loads return sooner
typedef __attribute__((address_space(4))) const uint32_t cword_t;

template <typename D>
__device__ __forceinline__ D scalar_desc(const D *tab, int f) {
    static_assert(sizeof(D) % 4 == 0, "whole words");
    const cword_t *src = (const cword_t *)(tab + f);
    D d;
    uint32_t *dst = (uint32_t *)&d;
#pragma unroll
    for (int q = 0; q < (int)(sizeof(D) / 4); q++) dst[q] = src[q];
    return d;
}

__device__ __forceinline__ FilmDev film_desc(const FilmDev *films, int f) { return scalar_desc(films, f); }

__device__ __forceinline__ int4 block_entry(const int4 *tab, int b) {
    const cword_t *src = (const cword_t *)(tab + b);
    return make_int4((int)src[0], (int)src[1], (int)src[2], (int)src[3]);
}

// ---------------------------------------------------------------------------
// probes at an integer time (the probe launch, and the probe block of the
// merged H/M launch for the kinds that read neither H nor energy partials;
// the probe launch's mean-M tree and block_order_sums3 add the same values
// in the same grouping)
// ---------------------------------------------------------------------------
// whether a probe samples at the step in progress (its counter `step`), and
// the sample's index
__device__ __forceinline__ bool probe_due(const ProbeDev &P, long long step, long long &sample) {
    const long long ev = P.every > 1 ? P.every : 1;
    const long long ks = step - P.start + 1;
    if (ks % ev) return false;
    sample = ks / ev - 1;
    return true;
}

// the sums of three runs of partials (run w: nb[w] >= 1 values from
// part + b0[w]) as a 256-thread block reduces each run (thread t adds values
// t, t + 256, ... in order, then a halving tree), formed by one wavefront:
// lane t keeps the sums of threads t, t + 64, t + 128, t + 192 of all three
// runs (twelve independent loads per loop pass; an index past a run reads its
// last value and drops it), takes the tree's first two levels in registers
// and the rest by shuffles -- the same additions in the same grouping, with
// no LDS. Lane 0 holds the sums.
__device__ __forceinline__ void block_order_sums3(const double *part, const int *b0, const int *nb, double *out) {
    const int t = (int)threadIdx.x; // 0..63
    double s[3][4];
    for (int w = 0; w < 3; w++)
        for (int q = 0; q < 4; q++) s[w][q] = 0.0;
    const int nmax = max(nb[0], max(nb[1], nb[2]));
    for (int base = t; base < nmax; base += 256)
        for (int w = 0; w < 3; w++)
            for (int q = 0; q < 4; q++) {
                const int b = base + 64 * q;
                const bool in = b < nb[w];
                const double x = part[b0[w] + (in ? b : nb[w] - 1)];
                s[w][q] = in ? s[w][q] + x : s[w][q];
            }
    for (int w = 0; w < 3; w++) {
        double r = (s[w][0] + s[w][2]) + (s[w][1] + s[w][3]); // levels 128 and 64
        for (int st = 32; st > 0; st >>= 1) {
            const double o = __shfl_down(r, st, 64);
            if (t < st) r = r + o;
        }
        out[w] = r;
    }
}

// the values of such a probe in the merged H/M launch's probe block, formed
// by its first wavefront (the others take no part): the E component at its
// site, or the film's mean M from its film blocks' partial sums in block
// order; valid in lane 0
template <typename T>
__device__ __forceinline__ void probe_e_or_m_values(const KParams<T> &p, const ProbeDev &P, double *v) {
    if (P.kind == 0) {
        if (threadIdx.x == 0) v[0] = (double)ldz(p, p.E[P.field], P.i, P.j, P.k);
        return;
    }
    const FilmDev &F = p.films[P.film];
    double sum[3];
    block_order_sums3(p.partial, F.blk0, F.nblk, sum);
    for (int w = 0; w < 3; w++) v[w] = sum[w] / F.ncells;
}

// thread 0 stores a sample into the probe's ring and raises the non-finite
// flag
template <typename T>
__device__ __forceinline__ void probe_store(const KParams<T> &p, const ProbeDev &P, long long sample,
                                            const double *v) {
    if (threadIdx.x != 0) return;
    const long long slot = sample % P.cap;
    bool bad = false;
    for (int w = 0; w < P.nval; w++) {
        P.data[slot * P.nval + w] = v[w];
        if (!isfinite(v[w])) bad = true;
    }
    if (bad) atomicOr(p.flag, 1);
}

// a slot's row of the packed table (KParams::coefv), fetched with one or two
// 16-byte loads and served to e_apply as its table (the class argument is
// the row's own)
template <typename T>
struct CoefRow {
    T ca[3], cb[3];
    __device__ __forceinline__ void get(int, int C, T &a, T &b) const {
        a = ca[C];
        b = cb[C];
    }
};

template <typename T>
__device__ __forceinline__ CoefRow<T> coef_row(const T *v, int row) {
    CoefRow<T> r;
    if constexpr (sizeof(T) == 4) {
        const float4 a = *(const float4 *)(v + kCoefRow<float> * (long long)row);
        const float2 b = *(const float2 *)(v + kCoefRow<float> * (long long)row + 4);
        r.ca[0] = a.x;
        r.cb[0] = a.y;
        r.ca[1] = a.z;
        r.cb[1] = a.w;
        r.ca[2] = b.x;
        r.cb[2] = b.y;
    } else {
        const double2 *q = (const double2 *)(v + kCoefRow<double> * (long long)row);
        const double2 a = q[0], b = q[1], c = q[2];
        r.ca[0] = a.x;
        r.cb[0] = a.y;
        r.ca[1] = b.x;
        r.cb[1] = b.y;
        r.ca[2] = c.x;
        r.cb[2] = c.y;
    }
    return r;
}

// is the face of family c at slot idx (folded) a magnetic site of a film?
template <typename T>
__device__ __forceinline__ bool face_is_magnetic(const KParams<T> &p, int c, const int *idx) {
    for (int f = 0; f < p.nfilm; f++) {
        const FilmDev &F = p.films[f];
        const int r0 = idx[0] - F.b0[0], r1 = idx[1] - F.b0[1], r2 = idx[2] - F.b0[2];
        if (r0 >= 0 && r0 < F.bn[0] && r1 >= 0 && r1 < F.bn[1] && r2 >= 0 && r2 < F.bn[2]) {
            const long long l = (long long)r0 + (long long)F.bn[0] * ((long long)r1 + (long long)F.bn[1] * r2);
            return F.prm[(c * 3) * F.ns + l] > 0.0;
        }
    }
    return false;
}

} // namespace mpx
