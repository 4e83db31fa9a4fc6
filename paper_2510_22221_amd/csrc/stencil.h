// stencil.h -- point updates shared by the step passes: the E full step of
// one edge and the merged pair of H/M half steps of one non-magnetic face.
//
// Scheme (arXiv:2510.22221, Methods, "Numerical Model"): E <- ca E + cb
// (curl H - J), ca and cb from the edge's mean eps and sigma (the E update
// that follows eq. iterate_H); H <- H - dt/(2 mu0) curl E per half step
// (eq. iterate_H with M = 0).  Every value follows the operation sequence of
// the plain definition (the library is built without FP contraction), so the
// float64 results of all passes are bitwise equal.
#pragma once

#include "device_common.h"

namespace mpx {

constexpr int kMixed = 255;

// coefficient table of edges whose four cells share one id, staged in LDS;
// PEC ids hold ca = cb = 0 (the edge stays zero)
template <typename T>
struct CoefLds {
    T ca[256], cb[256];
};

template <typename T>
__device__ __forceinline__ void stage_coef(const KParams<T> &p, CoefLds<T> &L, int tid, int nthreads) {
    for (int q = tid; q < 256; q += nthreads) {
        const CoefDev<T> cf = p.coef[q];
        L.ca[q] = cf.pec ? T(0) : cf.ca;
        L.cb[q] = cf.pec ? T(0) : cf.cb;
    }
}

template <typename T>
struct CaCb {
    T ca, cb;
    int pec;
};

// ca, cb of an edge of component C at slot idx (folded) whose four cells do
// not share one id: the cells at (C1, C2) offsets (-1,-1), (-1,0), (0,-1),
// (0,0), averaged in that order
// (out of line, with scalar arguments: rare, and kept out of the march's code)
template <typename T, int C>
__device__ __noinline__ CaCb<T> mixed_coef(const uint8_t *gid, const MatDev *gmat, int n0, int n1, int n2, int px,
                                           int per0, int per1, int per2, double eps0, double dt, double inv_dt, int i,
                                           int j, int k) {
    constexpr int C1 = (C + 1) % 3, C2 = (C + 2) % 3;
    const int idx[3] = {i, j, k};
    const int n[3] = {n0, n1, n2}, per[3] = {per0, per1, per2};
    int m[4];
#pragma unroll
    for (int u = 0; u < 2; u++)
#pragma unroll
        for (int v = 0; v < 2; v++) {
            int q[3] = {idx[0], idx[1], idx[2]};
            q[C1] -= 1 - u;
            q[C2] -= 1 - v;
            for (int a = 0; a < 3; a++) q[a] = fold(q[a], n[a], per[a]);
            m[2 * u + v] = gid[(long long)q[0] + (long long)px * ((long long)q[1] + (long long)n1 * q[2])];
        }
    CaCb<T> r;
    const MatDev &A0 = gmat[m[0]], &A1 = gmat[m[1]], &A2 = gmat[m[2]], &A3 = gmat[m[3]];
    r.pec = (A0.is_pec || A1.is_pec || A2.is_pec || A3.is_pec) ? 1 : 0;
    if constexpr (sizeof(T) == 8) {
        double se = 0.0, ss = 0.0;
        se += A0.eps_r;
        ss += A0.sigma;
        se += A1.eps_r;
        ss += A1.sigma;
        se += A2.eps_r;
        ss += A2.sigma;
        se += A3.eps_r;
        ss += A3.sigma;
        const double eps = eps0 * (se / 4);
        const double sig = ss / 4;
        const double den = sig / 2.0 + eps / dt;
        r.ca = -(sig / 2.0 - eps / dt) / den;
        r.cb = 1.0 / den;
    } else {
        // float32 fields: the float64 sequence rounded once, as in the table
        double se = 0.0, ss = 0.0;
        se += A0.eps_r;
        ss += A0.sigma;
        se += A1.eps_r;
        ss += A1.sigma;
        se += A2.eps_r;
        ss += A2.sigma;
        se += A3.eps_r;
        ss += A3.sigma;
        const double eps = eps0 * (se / 4);
        const double sig = ss / 4;
        const double den = sig / 2.0 + eps / dt;
        r.ca = (float)(-(sig / 2.0 - eps / dt) / den);
        r.cb = (float)(1.0 / den);
        (void)inv_dt;
    }
    return r;
}

// E^{n+1} of component C at raw position (gi, gj, gk) (possibly one past the
// domain on a periodic axis), given E^n, the class byte of its slot and the
// two raw curl differences d1 (along C1) and d2 (along C2).  `own`: this
// thread owns the edge and writes its E-type psi.
// PSI_INPLACE: the E-type psi live in one buffer (separate-pass schedule)
template <typename T, int C, bool WALL, bool PSI_INPLACE = false>
__device__ __forceinline__ T e_upd(const KParams<T> &p, const CoefLds<T> &L, int gi, int gj, int gk, int cls,
                                   T eold, T d1, T d2, bool tpml, bool tsrc, long long step, bool own) {
    constexpr int C1 = (C + 1) % 3, C2 = (C + 2) % 3;
    int idx[3] = {gi, gj, gk};
    if constexpr (WALL) {
#pragma unroll
        for (int a = 0; a < 3; a++) {
            if (p.per[a]) {
                if (idx[a] > p.n[a]) return T(0); // beyond a partial tile; never stored
                if (idx[a] == p.n[a]) idx[a] = 0;
            } else {
                if (a != C && idx[a] == 0) return T(0); // tangential to a wall
                if (idx[a] >= p.n[a]) return T(0);      // on the far wall (not stored)
            }
        }
    }
    T ca, cb;
    if (cls != kMixed) {
        ca = L.ca[cls];
        cb = L.cb[cls];
    } else {
        const CaCb<T> r = mixed_coef<T, C>(p.id, p.mat, p.n[0], p.n[1], p.n[2], p.px, p.per[0], p.per[1], p.per[2],
                                           p.eps0, p.dt, p.inv_dt, idx[0], idx[1], idx[2]);
        ca = r.pec ? T(0) : r.ca;
        cb = r.pec ? T(0) : r.cb;
    }
    // a PEC edge (cb = 0) stays zero and keeps its psi
    if (tpml && cb != T(0)) {
        const int a1 = idx[C1], a2 = idx[C2];
        if (p.psiE[C][C1] && (a1 < p.nlo[C1] || a1 >= p.n[C1] - p.nhi[C1])) {
            const long long qq = p.psi_index(C1, idx);
            const T ps = p.bE[C1][a1] * p.psiE[C][C1][qq] + p.cE[C1][a1] * d1;
            if (own) (PSI_INPLACE ? p.psiE : p.psiEb)[C][C1][qq] = ps;
            d1 += ps;
        }
        if (p.psiE[C][C2] && (a2 < p.nlo[C2] || a2 >= p.n[C2] - p.nhi[C2])) {
            const long long qq = p.psi_index(C2, idx);
            const T ps = p.bE[C2][a2] * p.psiE[C][C2][qq] + p.cE[C2][a2] * d2;
            if (own) (PSI_INPLACE ? p.psiE : p.psiEb)[C][C2][qq] = ps;
            d2 += ps;
        }
    }
    T x = d1 - d2;
    if (tsrc) {
        double J = 0.0;
        for (int s = 0; s < p.nsrc; s++) {
            const SrcDev &S = p.srcs[s]; // device copy: no dynamic index into the kernel argument
            if (S.comp != C) continue;
            if (idx[0] < S.box[0] || idx[0] >= S.box[0] + S.box[3] || idx[1] < S.box[1] ||
                idx[1] >= S.box[1] + S.box[4] || idx[2] < S.box[2] || idx[2] >= S.box[2] + S.box[5])
                continue;
            if (step < S.n) J += S.table[step];
        }
        // (x - 0) is x bitwise, so subtracting only here matches the plain form
        x = x - T(J);
    }
    return ca * eold + cb * x;
}

// NHALF consecutive H/M half steps with the same E (2: the merged pair
// around an integer time, 1: a bracket half step) of component C at the
// owned slot idx (folded), given the raw differences of E
template <typename T, int C, int NHALF = 2>
__device__ __forceinline__ T h_upd(const KParams<T> &p, const int *idx, T h, T d1r, T d2r, bool tpml) {
    constexpr int C1 = (C + 1) % 3, C2 = (C + 2) % 3;
    bool s1 = false, s2 = false;
    long long q1 = 0, q2 = 0;
    T ps1 = T(0), ps2 = T(0);
    const int a1 = idx[C1], a2 = idx[C2];
    if (tpml) {
        s1 = p.psiH[C][C1] && (a1 < p.nlo[C1] || a1 >= p.n[C1] - p.nhi[C1]);
        s2 = p.psiH[C][C2] && (a2 < p.nlo[C2] || a2 >= p.n[C2] - p.nhi[C2]);
        if (s1) {
            q1 = p.psi_index(C1, idx);
            ps1 = p.psiH[C][C1][q1];
        }
        if (s2) {
            q2 = p.psi_index(C2, idx);
            ps2 = p.psiH[C][C2][q2];
        }
    }
#pragma unroll
    for (int hs = 0; hs < NHALF; hs++) {
        T d1 = d1r, d2 = d2r;
        if (s1) {
            ps1 = p.bH[C1][a1] * ps1 + p.cH[C1][a1] * d1;
            d1 += ps1;
        }
        if (s2) {
            ps2 = p.bH[C2][a2] * ps2 + p.cH[C2][a2] * d2;
            d2 += ps2;
        }
        h = h - p.hc * (d1 - d2);
    }
    if (s1) p.psiH[C][C1][q1] = ps1;
    if (s2) p.psiH[C][C2][q2] = ps2;
    return h;
}

// class byte at raw (i, j, k): folded on periodic axes, "mixed" outside
template <typename T>
__device__ __forceinline__ int ldcls(const KParams<T> &p, int i, int j, int k) {
    const int ii = fold(i, p.n[0], p.per[0]), jj = fold(j, p.n[1], p.per[1]), kk = fold(k, p.n[2], p.per[2]);
    if (ii < 0 || jj < 0 || kk < 0) return kMixed;
    return p.cls[p.slot(ii, jj, kk)];
}

} // namespace mpx
