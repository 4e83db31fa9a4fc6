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
