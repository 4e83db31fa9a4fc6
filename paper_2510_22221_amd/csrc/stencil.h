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

// coefficient table by slot class and edge component, staged in LDS; PEC
// edges hold ca = cb = 0 (the edge stays zero)
template <typename T>
struct CoefLds {
    T ca[kCoefEntries], cb[kCoefEntries];
    __device__ __forceinline__ void get(int cls, int C, T &a, T &b) const {
        a = ca[kCoefPerClass * cls + C];
        b = cb[kCoefPerClass * cls + C];
    }
};

// the same table read straight from device memory (the host stores PEC
// entries as ca = cb = 0)
template <typename T>
struct CoefMem {
    const CoefDev<T> *c;
    __device__ __forceinline__ void get(int cls, int C, T &a, T &b) const {
        a = c[kCoefPerClass * cls + C].ca;
        b = c[kCoefPerClass * cls + C].cb;
    }
};

template <typename T>
__device__ __forceinline__ void stage_coef(const KParams<T> &p, CoefLds<T> &L, int tid, int nthreads) {
    for (int q = tid; q < kCoefEntries; q += nthreads) {
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

// CPML state of one component at one site for its two derivative axes:
// slab membership, slab-compact index, psi and the recursion coefficients.
// Loaded before any store of a pass (so every load of a thread is in flight
// at once), applied, then stored.
template <typename T>
struct Psi2 {
    bool s1 = false, s2 = false, upd = false;
    long long q1 = 0, q2 = 0;
    T ps1 = T(0), ps2 = T(0), b1 = T(0), c1 = T(0), b2 = T(0), c2 = T(0);
};

// E: the E-type psi (E = true) or H-type psi of component C at the folded
// site idx.  A slot's psi is touched once per pass: the y- and z-slab arrays
// load and store it non-temporal; the x-slab arrays keep the default policy
// (a row's few slab values share cache lines with the next row's, which
// another tile reads)
template <typename T, int C, bool E>
__device__ __forceinline__ Psi2<T> psi_load(const KParams<T> &p, const int *idx) {
    constexpr int C1 = (C + 1) % 3, C2 = (C + 2) % 3;
    Psi2<T> r;
    T *const *arr = E ? p.psiE[C] : p.psiH[C];
    const T *const *bt = E ? p.bE : p.bH;
    const T *const *ct = E ? p.cE : p.cH;
    const int a1 = idx[C1], a2 = idx[C2];
    r.s1 = arr[C1] && (a1 < p.nlo[C1] || a1 >= p.n[C1] - p.nhi[C1]);
    r.s2 = arr[C2] && (a2 < p.nlo[C2] || a2 >= p.n[C2] - p.nhi[C2]);
    if (r.s1) {
        r.q1 = p.psi_index(C1, idx);
        r.ps1 = C1 == 0 ? arr[C1][r.q1] : __builtin_nontemporal_load(arr[C1] + r.q1);
        r.b1 = bt[C1][a1];
        r.c1 = ct[C1][a1];
    }
    if (r.s2) {
        r.q2 = p.psi_index(C2, idx);
        r.ps2 = C2 == 0 ? arr[C2][r.q2] : __builtin_nontemporal_load(arr[C2] + r.q2);
        r.b2 = bt[C2][a2];
        r.c2 = ct[C2][a2];
    }
    return r;
}

template <typename T, int C>
__device__ __forceinline__ void psi_store(T *const *arr, const Psi2<T> &r) {
    constexpr int C1 = (C + 1) % 3, C2 = (C + 2) % 3;
    if (!r.upd) return;
    if (r.s1) {
        if (C1 == 0)
            arr[C1][r.q1] = r.ps1;
        else
            __builtin_nontemporal_store(r.ps1, arr[C1] + r.q1);
    }
    if (r.s2) {
        if (C2 == 0)
            arr[C2][r.q2] = r.ps2;
        else
            __builtin_nontemporal_store(r.ps2, arr[C2] + r.q2);
    }
}

// the E edge of component C at raw position (gi, gj, gk) (possibly one past
// the domain on a periodic axis): false when it lies on a wall (held at
// zero) or beyond a partial tile; idx receives the folded position
template <typename T, int C, bool WALL>
__device__ __forceinline__ bool e_site(const KParams<T> &p, int gi, int gj, int gk, int *idx) {
    idx[0] = gi;
    idx[1] = gj;
    idx[2] = gk;
    if constexpr (WALL) {
#pragma unroll
        for (int a = 0; a < 3; a++) {
            if (p.per[a]) {
                if (idx[a] > p.n[a]) return false; // beyond a partial tile; never stored
                if (idx[a] == p.n[a]) idx[a] = 0;
            } else {
                if (a != C && idx[a] == 0) return false; // tangential to a wall
                if (idx[a] >= p.n[a]) return false;      // on the far wall (not stored)
            }
        }
    }
    return true;
}

// E^{n+1} of component C at the folded site idx (a valid edge), given E^n,
// the class byte of its slot, the two raw curl differences d1 (along C1) and
// d2 (along C2) and its loaded CPML state (advanced here; r.upd tells the
// caller to store it: a PEC edge, cb = 0, stays zero and keeps its psi)
// (MIXED = false: the caller guarantees a table class, no mixed path)
template <typename T, int C, class TAB, bool MIXED = true>
__device__ __forceinline__ T e_apply(const KParams<T> &p, const TAB &L, const int *idx, int cls, T eold, T d1, T d2,
                                     Psi2<T> &r, bool tsrc, long long step) {
    T ca, cb;
    if (!MIXED || cls != kMixed) {
        L.get(cls, C, ca, cb);
    } else {
        const CaCb<T> m = mixed_coef<T, C>(p.id, p.mat, p.n[0], p.n[1], p.n[2], p.px, p.per[0], p.per[1], p.per[2],
                                           p.eps0, p.dt, p.inv_dt, idx[0], idx[1], idx[2]);
        ca = m.pec ? T(0) : m.ca;
        cb = m.pec ? T(0) : m.cb;
    }
    r.upd = cb != T(0);
    if (r.upd) {
        if (r.s1) {
            r.ps1 = r.b1 * r.ps1 + r.c1 * d1;
            d1 += r.ps1;
        }
        if (r.s2) {
            r.ps2 = r.b2 * r.ps2 + r.c2 * d2;
            d2 += r.ps2;
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

// the whole E update of one edge (load psi, apply, store psi).
// PSI_INPLACE: the E-type psi live in one buffer (separate-pass schedule);
// `own`: this thread owns the edge and writes its psi.
template <typename T, int C, bool WALL, bool PSI_INPLACE = false, class TAB = CoefLds<T>, bool MIXED = true>
__device__ __forceinline__ T e_upd(const KParams<T> &p, const TAB &L, int gi, int gj, int gk, int cls,
                                   T eold, T d1, T d2, bool tpml, bool tsrc, long long step, bool own) {
    int idx[3];
    if (!e_site<T, C, WALL>(p, gi, gj, gk, idx)) return T(0);
    Psi2<T> r;
    if (tpml) r = psi_load<T, C, true>(p, idx);
    const T e = e_apply<T, C, TAB, MIXED>(p, L, idx, cls, eold, d1, d2, r, tsrc, step);
    if (own) psi_store<T, C>(PSI_INPLACE ? p.psiE[C] : p.psiEb[C], r);
    return e;
}

// NHALF consecutive H/M half steps with the same E (2: the merged pair
// around an integer time, 1: a bracket half step) of component C, given the
// raw differences of E and its loaded CPML state (advanced here)
template <typename T, int C, int NHALF>
__device__ __forceinline__ T h_apply(const KParams<T> &p, T h, T d1r, T d2r, Psi2<T> &r) {
#pragma unroll
    for (int hs = 0; hs < NHALF; hs++) {
        T d1 = d1r, d2 = d2r;
        if (r.s1) {
            r.ps1 = r.b1 * r.ps1 + r.c1 * d1;
            d1 += r.ps1;
        }
        if (r.s2) {
            r.ps2 = r.b2 * r.ps2 + r.c2 * d2;
            d2 += r.ps2;
        }
        h = h - p.hc * (d1 - d2);
    }
    r.upd = true;
    return h;
}

// the whole H update of one owned face (folded idx)
template <typename T, int C, int NHALF = 2>
__device__ __forceinline__ T h_upd(const KParams<T> &p, const int *idx, T h, T d1r, T d2r, bool tpml) {
    Psi2<T> r;
    if (tpml) r = psi_load<T, C, false>(p, idx);
    h = h_apply<T, C, NHALF>(p, h, d1r, d2r, r);
    psi_store<T, C>(p.psiH[C], r);
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
