// kernels.hip -- gfx950 device code of libmpx: the Yee curl updates, the
// CPML recursions, the soft source, the trapezoidal LLG site solve and the
// probe / energy reductions.
//
// Scheme: arXiv:2510.22221, Methods, "Numerical Model".
//   H/M half step: B^ = H + M, B^* = B^ - dt/(2 mu0) curl E (eq. iterate_H);
//     non-magnetic faces keep H = B^*; magnetic faces solve the trapezoidal
//     LLG (eqs. llg_tra4-llg_tra6) at its fixed point, normalise to Ms and
//     set H = B^*_c - M_c.
//   E step: E <- ca E + cb (curl H - J), ca, cb from eps and sigma of the
//     edge (the semi-implicit E update closing that subsection).
//
// Layout: every field component lives on an nx*ny*nz slot lattice, x fastest
// with a padded pitch; slot (i,j,k) holds the Yee site with natural index
// (i,j,k).  Sites with natural index N along a non-periodic axis lie on the
// domain wall and are identically zero, so they are not stored.
//
// Arithmetic order: the float64 instantiation evaluates every stored value
// with the same sequence of IEEE operations as the plain definition (the
// library is built with -ffp-contract=off), so repeated runs, tile shapes and
// the fused pass all give bitwise identical float64 results.
#include "mpx_internal.h"

namespace mpx {

__device__ __forceinline__ int fold(int i, int n, int per) {
    if (per) {
        if (i < 0) i += n;
        if (i >= n) i -= n;
        return i;
    }
    return (i < 0 || i >= n) ? -1 : i;
}

template <typename T>
__device__ __forceinline__ T ldz(const KParams<T> &p, const T *a, int i, int j, int k) {
    int ii = fold(i, p.n[0], p.per[0]), jj = fold(j, p.n[1], p.per[1]), kk = fold(k, p.n[2], p.per[2]);
    if (ii < 0 || jj < 0 || kk < 0) return T(0);
    return a[p.slot(ii, jj, kk)];
}

__device__ __forceinline__ int cell_id(const int *n, const int *per, int px, const uint8_t *id, int i, int j,
                                       int k) {
    int ii = fold(i, n[0], per[0]), jj = fold(j, n[1], per[1]), kk = fold(k, n[2], per[2]);
    if (ii < 0 || jj < 0 || kk < 0) return -1;
    return id[(long long)ii + (long long)px * ((long long)jj + (long long)n[1] * kk)];
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

// ---------------------------------------------------------------------------
// magnetic-face test: the face of family c at slot idx is magnetic when it
// lies in a film's site box and one of the two cells sharing it has Ms > 0
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ int film_of_site(const KParams<T> &p, int c, const int *idx) {
    for (int f = 0; f < p.nfilm; f++) {
        const FilmDev &F = p.films[f];
        if (idx[0] >= F.b0[0] && idx[0] < F.b0[0] + F.bn[0] && idx[1] >= F.b0[1] && idx[1] < F.b0[1] + F.bn[1] &&
            idx[2] >= F.b0[2] && idx[2] < F.b0[2] + F.bn[2]) {
            int lo[3] = {idx[0], idx[1], idx[2]};
            lo[c] -= 1;
            int m0 = cell_id(p.n, p.per, p.px, p.id, lo[0], lo[1], lo[2]);
            int m1 = cell_id(p.n, p.per, p.px, p.id, idx[0], idx[1], idx[2]);
            bool mag = (m0 >= 0 && p.mat[m0].Ms > 0.0) || (m1 >= 0 && p.mat[m1].Ms > 0.0);
            return mag ? f : -1;
        }
    }
    return -1;
}

// ---------------------------------------------------------------------------
// bulk H/M pass for non-magnetic faces: NHALF consecutive half steps with the
// same E (1 = a bracket half step, 2 = the merged pair around an integer time)
// ---------------------------------------------------------------------------
template <typename T, int NHALF>
__global__ void __launch_bounds__(256) k_hbulk(KParams<T> p, int inc_step) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (inc_step && i == 0 && j == 0 && k == 0) p.step[0] = p.step[0] + 1;
    if (i >= p.n[0] || j >= p.n[1]) return;
    const long long q = p.slot(i, j, k);
    const int idx[3] = {i, j, k};
    for (int c = 0; c < 3; c++) {
        if (p.nfilm && film_of_site(p, c, idx) >= 0) continue;
        const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        int u1[3] = {i, j, k}, u2[3] = {i, j, k};
        u1[c1] += 1;
        u2[c2] += 1;
        const T e2a = p.E[c2][q];
        const T e2b = ldz(p, p.E[c2], u1[0], u1[1], u1[2]);
        const T e1a = p.E[c1][q];
        const T e1b = ldz(p, p.E[c1], u2[0], u2[1], u2[2]);
        const T d1r = dif(e2b, e2a, p.dT[c1], p.invd[c1]);
        const T d2r = dif(e1b, e1a, p.dT[c2], p.invd[c2]);
        // H_c sits at half positions along c1 and c2
        const int a1 = idx[c1], a2 = idx[c2];
        const bool s1 = p.psiH[c][c1] && (a1 < p.nlo[c1] || a1 >= p.n[c1] - p.nhi[c1]);
        const bool s2 = p.psiH[c][c2] && (a2 < p.nlo[c2] || a2 >= p.n[c2] - p.nhi[c2]);
        long long q1 = 0, q2 = 0;
        T ps1 = T(0), ps2 = T(0);
        if (s1) {
            q1 = p.psi_index(c1, idx);
            ps1 = p.psiH[c][c1][q1];
        }
        if (s2) {
            q2 = p.psi_index(c2, idx);
            ps2 = p.psiH[c][c2][q2];
        }
        T h = p.H[c][q];
#pragma unroll
        for (int hs = 0; hs < NHALF; hs++) {
            T d1 = d1r, d2 = d2r;
            if (s1) {
                ps1 = p.bH[c1][a1] * ps1 + p.cH[c1][a1] * d1;
                d1 += ps1;
            }
            if (s2) {
                ps2 = p.bH[c2][a2] * ps2 + p.cH[c2][a2] * d2;
                d2 += ps2;
            }
            h = h - p.hc * (d1 - d2);
        }
        p.H[c][q] = h;
        if (s1) p.psiH[c][c1][q1] = ps1;
        if (s2) p.psiH[c][c2][q2] = ps2;
    }
}

// ---------------------------------------------------------------------------
// edge coefficients from the per-cell material ids: eps and sigma are the
// means over the four cells sharing the edge, the edge is PEC if any is PEC
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ bool edge_coef(const KParams<T> &p, int c, const int *idx, T &ca, T &cb) {
    const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
    double se = 0.0, ss = 0.0;
    int cnt = 0;
    bool pec = false;
    for (int u = -1; u <= 0; u++)
        for (int v = -1; v <= 0; v++) {
            int cc[3];
            cc[c] = idx[c];
            cc[c1] = idx[c1] + u;
            cc[c2] = idx[c2] + v;
            int m = cell_id(p.n, p.per, p.px, p.id, cc[0], cc[1], cc[2]);
            if (m < 0) continue;
            se += p.mat[m].eps_r;
            ss += p.mat[m].sigma;
            pec = pec || p.mat[m].is_pec;
            cnt++;
        }
    if (pec || cnt == 0) return false;
    if constexpr (sizeof(T) == 8) {
        const double eps = p.eps0 * (se / cnt);
        const double sig = ss / cnt;
        const double den = sig / 2.0 + eps / p.dt;
        ca = -(sig / 2.0 - eps / p.dt) / den;
        cb = 1.0 / den;
    } else {
        const float eps = float(p.eps0) * (float(se) / float(cnt));
        const float sig = float(ss) / float(cnt);
        const float den = sig * 0.5f + eps * float(p.inv_dt);
        const float rden = 1.0f / den;
        ca = -(sig * 0.5f - eps * float(p.inv_dt)) * rden;
        cb = rden;
    }
    return true;
}

// ---------------------------------------------------------------------------
// E pass: full step on every non-PEC edge, CPML psi in the slabs, soft source
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_epass(KParams<T> p) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= p.n[0] || j >= p.n[1]) return;
    const long long q = p.slot(i, j, k);
    const int idx[3] = {i, j, k};
    const long long step = p.step[0];
    for (int c = 0; c < 3; c++) {
        const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        // tangential to a non-periodic wall: held at zero
        if ((!p.per[c1] && idx[c1] == 0) || (!p.per[c2] && idx[c2] == 0)) continue;
        T ca, cb;
        if (!edge_coef(p, c, idx, ca, cb)) continue;
        int l1[3] = {i, j, k}, l2[3] = {i, j, k};
        l1[c1] -= 1;
        l2[c2] -= 1;
        const T h2a = p.H[c2][q];
        const T h2b = ldz(p, p.H[c2], l1[0], l1[1], l1[2]);
        const T h1a = p.H[c1][q];
        const T h1b = ldz(p, p.H[c1], l2[0], l2[1], l2[2]);
        T d1 = dif(h2a, h2b, p.dT[c1], p.invd[c1]);
        T d2 = dif(h1a, h1b, p.dT[c2], p.invd[c2]);
        // E_c sits at integer positions along c1 and c2
        const int a1 = idx[c1], a2 = idx[c2];
        if (p.psiE[c][c1] && (a1 < p.nlo[c1] || a1 >= p.n[c1] - p.nhi[c1])) {
            const long long qq = p.psi_index(c1, idx);
            const T ps = p.bE[c1][a1] * p.psiE[c][c1][qq] + p.cE[c1][a1] * d1;
            p.psiE[c][c1][qq] = ps;
            d1 += ps;
        }
        if (p.psiE[c][c2] && (a2 < p.nlo[c2] || a2 >= p.n[c2] - p.nhi[c2])) {
            const long long qq = p.psi_index(c2, idx);
            const T ps = p.bE[c2][a2] * p.psiE[c][c2][qq] + p.cE[c2][a2] * d2;
            p.psiE[c][c2][qq] = ps;
            d2 += ps;
        }
        double J = 0.0;
        for (int s = 0; s < p.nsrc; s++) {
            const SrcDev &S = p.src[s];
            if (S.comp != c) continue;
            if (i < S.box[0] || i >= S.box[0] + S.box[3] || j < S.box[1] || j >= S.box[1] + S.box[4] ||
                k < S.box[2] || k >= S.box[2] + S.box[5])
                continue;
            if (step < S.n) J += S.table[step];
        }
        p.E[c][q] = ca * p.E[c][q] + cb * ((d1 - d2) - T(J));
    }
}

// ---------------------------------------------------------------------------
// film half step (float64 throughout)
//   phase 1: reads the state (H, M); writes the scratch (H1, M1)
//   phase 2: reads the scratch for magnetic faces and recomputes the first
//            half step on the fly for non-magnetic ones; writes the state
// ---------------------------------------------------------------------------
struct SiteRef {
    int film;
    long long l; // local index in the film's site box
};

template <typename T>
__device__ __forceinline__ long long film_local(const FilmDev &F, const int *idx, bool &inside) {
    int r[3];
    for (int a = 0; a < 3; a++) {
        r[a] = idx[a] - F.b0[a];
        if (r[a] < 0 || r[a] >= F.bn[a]) {
            inside = false;
            return 0;
        }
    }
    inside = true;
    return (long long)r[0] + (long long)F.bn[0] * ((long long)r[1] + (long long)F.bn[1] * r[2]);
}

template <typename T>
__device__ __forceinline__ void site_params(const KParams<T> &p, int c, const int *idx, double &ms, double &al,
                                            double &ga) {
    double sm = 0.0, sa = 0.0, sg = 0.0;
    int cnt = 0, nm = 0;
    for (int u = -1; u <= 0; u++) {
        int cc[3] = {idx[0], idx[1], idx[2]};
        cc[c] += u;
        int m = cell_id(p.n, p.per, p.px, p.id, cc[0], cc[1], cc[2]);
        if (m < 0) continue;
        cnt++;
        sm += p.mat[m].Ms;
        if (p.mat[m].Ms > 0) {
            nm++;
            sa += p.mat[m].alpha;
            sg += p.mat[m].gamma_abs;
        }
    }
    ms = cnt ? sm / cnt : 0.0;
    al = nm ? sa / nm : 0.0;
    ga = nm ? sg / nm : 0.0;
}

// (curl E)_c parts at the H_c site idx, in float64
template <typename T>
__device__ __forceinline__ void curl_e64(const KParams<T> &p, int c, const int *idx, double &d1, double &d2) {
    const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
    int u1[3] = {idx[0], idx[1], idx[2]}, u2[3] = {idx[0], idx[1], idx[2]};
    u1[c1] += 1;
    u2[c2] += 1;
    const double e2a = (double)ldz(p, p.E[c2], idx[0], idx[1], idx[2]);
    const double e2b = (double)ldz(p, p.E[c2], u1[0], u1[1], u1[2]);
    const double e1a = (double)ldz(p, p.E[c1], idx[0], idx[1], idx[2]);
    const double e1b = (double)ldz(p, p.E[c1], u2[0], u2[1], u2[2]);
    d1 = (e2b - e2a) / p.d[c1];
    d2 = (e1b - e1a) / p.d[c2];
}

// B^ and B^* at the face of family cq at idx (folded), for film f
template <typename T>
__device__ __forceinline__ void bhat(const KParams<T> &p, int phase, int f, int cq, const int *idx, double &bn,
                                     double &bs) {
    if (idx[0] < 0 || idx[1] < 0 || idx[2] < 0) { // outside the domain (cannot happen for the
        bn = bs = 0.0;                             // film placements set_materials accepts)
        return;
    }
    double d1, d2;
    curl_e64(p, cq, idx, d1, d2);
    const FilmDev &F = p.films[f];
    bool inside;
    const long long l = film_local<T>(F, idx, inside);
    bool mag = false;
    if (inside) {
        double ms, al, ga;
        site_params(p, cq, idx, ms, al, ga);
        mag = ms > 0.0;
    }
    double b;
    if (mag) {
        if (phase == 1)
            b = (double)p.H[cq][p.slot(idx[0], idx[1], idx[2])] + F.M[(cq * 3 + cq) * F.ns + l];
        else
            b = F.H1[cq * F.ns + l] + F.M1[(cq * 3 + cq) * F.ns + l];
    } else {
        double h = (double)p.H[cq][p.slot(idx[0], idx[1], idx[2])];
        if (phase == 2) h = h - p.hcd * (d1 - d2);
        b = h + 0.0;
    }
    bn = b;
    bs = b - p.hcd * (d1 - d2);
}

__device__ __forceinline__ void cross3(const double *a, const double *b, double *r) {
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}

__device__ __forceinline__ double dot3(const double *a, const double *b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

template <typename T>
__global__ void __launch_bounds__(256) k_film(KParams<T> p, int phase) {
    __shared__ double red[256];
    const int4 bt = p.blocktab[blockIdx.x]; // film, family, first local index
    const int f = bt.x, c = bt.y;
    const FilmDev &F = p.films[f];
    const long long l = (long long)bt.z + threadIdx.x;
    double own = 0.0;
    if (l < F.ns) {
        int idx[3];
        idx[0] = F.b0[0] + (int)(l % F.bn[0]);
        idx[1] = F.b0[1] + (int)((l / F.bn[0]) % F.bn[1]);
        idx[2] = F.b0[2] + (int)(l / ((long long)F.bn[0] * F.bn[1]));
        double ms, al, ga;
        site_params(p, c, idx, ms, al, ga);
        if (ms > 0.0) {
            double bn, bs;
            bhat(p, phase, f, c, idx, bn, bs);
            double P[3], Q[3], M[3];
            P[c] = bs;
            Q[c] = bn;
            for (int cp = 0; cp < 3; cp++) {
                if (cp == c) continue;
                // I_{c'}: mean of the four nearest family-c' faces, indices
                // {idx_c - 1, idx_c} along c and {idx_c', idx_c' + 1} along c'
                double vn[2][2], vs[2][2];
                for (int u = 0; u < 2; u++)
                    for (int v = 0; v < 2; v++) {
                        int q[3] = {idx[0], idx[1], idx[2]};
                        q[c] += u - 1;
                        q[cp] += v;
                        for (int a = 0; a < 3; a++) q[a] = fold(q[a], p.n[a], p.per[a]);
                        bhat(p, phase, f, cp, q, vn[u][v], vs[u][v]);
                    }
                Q[cp] = ((vn[0][0] + vn[1][0]) + (vn[0][1] + vn[1][1])) * 0.25;
                P[cp] = ((vs[0][0] + vs[1][0]) + (vs[0][1] + vs[1][1])) * 0.25;
            }
            const double *Msrc = (phase == 1) ? F.M : F.M1;
            for (int w = 0; w < 3; w++) {
                P[w] += p.H0[w];
                Q[w] += p.H0[w];
                M[w] = Msrc[(c * 3 + w) * F.ns + l];
            }
            const double kk = p.kf * ga;
            // b = M^n - k (M^n x H_eff^n), with H_eff^n = Q - M^n
            double MxQ[3], b[3], a[3];
            cross3(M, Q, MxQ);
            for (int w = 0; w < 3; w++) b[w] = M[w] - kk * MxQ[w];
            // a at the fixed point: H_eff^{n+1} = P - M^{n+1}
            for (int w = 0; w < 3; w++) a[w] = -(kk * P[w] + (al / ms) * M[w]);
            // X = (b + (a.b) a - a x b) / (1 + |a|^2), then M' = Ms X/|X|
            double axb[3], X[3], Mn[3];
            cross3(a, b, axb);
            const double ab = dot3(a, b), aa = dot3(a, a);
            for (int w = 0; w < 3; w++) X[w] = (b[w] + ab * a[w] - axb[w]) / (1.0 + aa);
            const double nx = sqrt(dot3(X, X));
            for (int w = 0; w < 3; w++) Mn[w] = ms * X[w] / nx;
            const double hnew = bs - Mn[c];
            if (phase == 1) {
                for (int w = 0; w < 3; w++) F.M1[(c * 3 + w) * F.ns + l] = Mn[w];
                F.H1[c * F.ns + l] = hnew;
            } else {
                for (int w = 0; w < 3; w++) F.M[(c * 3 + w) * F.ns + l] = Mn[w];
                p.H[c][p.slot(idx[0], idx[1], idx[2])] = (T)hnew;
            }
            own = Mn[c];
        }
    }
    // block partial of the own component (mean-M probes)
    red[threadIdx.x] = own;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) p.partial[blockIdx.x] = red[0];
}

// copy the scratch of a single (bracket) half step into the state
template <typename T>
__global__ void __launch_bounds__(256) k_film_commit(KParams<T> p) {
    const int4 bt = p.blocktab[blockIdx.x];
    const int f = bt.x, c = bt.y;
    const FilmDev &F = p.films[f];
    const long long l = (long long)bt.z + threadIdx.x;
    if (l >= F.ns) return;
    int idx[3];
    idx[0] = F.b0[0] + (int)(l % F.bn[0]);
    idx[1] = F.b0[1] + (int)((l / F.bn[0]) % F.bn[1]);
    idx[2] = F.b0[2] + (int)(l / ((long long)F.bn[0] * F.bn[1]));
    double ms, al, ga;
    site_params(p, c, idx, ms, al, ga);
    if (!(ms > 0.0)) return;
    for (int w = 0; w < 3; w++) F.M[(c * 3 + w) * F.ns + l] = F.M1[(c * 3 + w) * F.ns + l];
    p.H[c][p.slot(idx[0], idx[1], idx[2])] = (T)F.H1[c * F.ns + l];
}

// ---------------------------------------------------------------------------
// probes at an integer time: after the E step and the first H/M half step of
// the merged pair (scratch holds H, M at that time for magnetic faces)
// ---------------------------------------------------------------------------
template <typename T>
__device__ double h_integer_time(const KParams<T> &p, int c, const int *idx) {
    const int f = p.nfilm ? film_of_site(p, c, idx) : -1;
    if (f >= 0) {
        const FilmDev &F = p.films[f];
        bool inside;
        const long long l = film_local<T>(F, idx, inside);
        return F.H1[c * F.ns + l];
    }
    const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
    int u1[3] = {idx[0], idx[1], idx[2]}, u2[3] = {idx[0], idx[1], idx[2]};
    u1[c1] += 1;
    u2[c2] += 1;
    const T d1 = dif(ldz(p, p.E[c2], u1[0], u1[1], u1[2]), ldz(p, p.E[c2], idx[0], idx[1], idx[2]), p.dT[c1],
                     p.invd[c1]);
    const T d2 = dif(ldz(p, p.E[c1], u2[0], u2[1], u2[2]), ldz(p, p.E[c1], idx[0], idx[1], idx[2]), p.dT[c2],
                     p.invd[c2]);
    const T h = ldz(p, p.H[c], idx[0], idx[1], idx[2]);
    return (double)(h - p.hc * (d1 - d2));
}

template <typename T>
__global__ void __launch_bounds__(256) k_probes(KParams<T> p) {
    __shared__ double red[256];
    const ProbeDev &P = p.probes[blockIdx.x];
    const long long step = p.step[0];
    double v[3] = {0.0, 0.0, 0.0};
    if (P.kind == 0) {
        if (threadIdx.x == 0) {
            const int idx[3] = {P.i, P.j, P.k};
            if (P.field < 3)
                v[0] = (double)ldz(p, p.E[P.field], P.i, P.j, P.k);
            else {
                // sites on an upper wall are not stored and are zero
                const int c = P.field - 3;
                bool wall = false;
                for (int a = 0; a < 3; a++)
                    if (idx[a] >= p.n[a]) wall = true;
                v[0] = wall ? 0.0 : h_integer_time(p, c, idx);
            }
        }
    } else if (P.kind == 1) {
        const FilmDev &F = p.films[P.film];
        for (int w = 0; w < 3; w++) {
            const int b0 = F.blk0[w], nb = F.nblk[w];
            double s = 0.0;
            for (int b = threadIdx.x; b < nb; b += blockDim.x) s += p.partial[b0 + b];
            red[threadIdx.x] = s;
            __syncthreads();
            for (int st = 128; st > 0; st >>= 1) {
                if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
                __syncthreads();
            }
            v[w] = red[0] / F.ncells;
            __syncthreads();
        }
    } else {
        const FilmDev &F = p.films[P.film];
        const long long ncell = (long long)F.cb[3] * F.cb[4] * F.cb[5];
        double s = 0.0;
        for (long long t = threadIdx.x; t < ncell; t += blockDim.x) {
            const int cc[3] = {F.cb[0] + (int)(t % F.cb[3]), F.cb[1] + (int)((t / F.cb[3]) % F.cb[4]),
                               F.cb[2] + (int)(t / ((long long)F.cb[3] * F.cb[4]))};
            const int m = cell_id(p.n, p.per, p.px, p.id, cc[0], cc[1], cc[2]);
            if (m < 0 || !(p.mat[m].Ms > 0.0)) continue;
            double we = 0.0, wh = 0.0;
            for (int c = 0; c < 3; c++) {
                const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
                double e2 = 0.0;
                for (int u = 0; u < 2; u++)
                    for (int vv = 0; vv < 2; vv++) {
                        int q[3] = {cc[0], cc[1], cc[2]};
                        q[c1] += u;
                        q[c2] += vv;
                        const double e = (double)ldz(p, p.E[c], q[0], q[1], q[2]);
                        e2 += e * e;
                    }
                we += e2 / 4.0;
                double h2 = 0.0;
                for (int u = 0; u < 2; u++) {
                    int q[3] = {cc[0], cc[1], cc[2]};
                    q[c] += u;
                    for (int a = 0; a < 3; a++) q[a] = fold(q[a], p.n[a], p.per[a]);
                    const double h = (q[0] < 0 || q[1] < 0 || q[2] < 0) ? 0.0 : h_integer_time(p, c, q);
                    h2 += h * h;
                }
                wh += h2 / 2.0;
            }
            s += 0.5 * p.eps0 * p.mat[m].eps_r * we + 0.5 * p.mu0 * wh;
        }
        red[threadIdx.x] = s;
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
            if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
            __syncthreads();
        }
        v[0] = red[0] * p.dV;
    }
    if (threadIdx.x == 0) {
        const long long slot = (step - P.start) % P.cap;
        bool bad = false;
        for (int w = 0; w < P.nval; w++) {
            P.data[slot * P.nval + w] = v[w];
            if (!isfinite(v[w])) bad = true;
        }
        if (bad) atomicOr(p.flag, 1);
    }
}

// ---------------------------------------------------------------------------
// discrete energy at an integer time: per-block partials of
// sum eps_e E^2, sum (H^2 - (hc curl E)^2) and sum H0_c M_c
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_energy(KParams<T> p, double *part) {
    __shared__ double red[3][256];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    const int t = threadIdx.x + blockDim.x * threadIdx.y;
    double we = 0.0, wh = 0.0;
    if (i < p.n[0] && j < p.n[1]) {
        const int idx[3] = {i, j, k};
        const long long q = p.slot(i, j, k);
        for (int c = 0; c < 3; c++) {
            const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
            if (!((!p.per[c1] && idx[c1] == 0) || (!p.per[c2] && idx[c2] == 0))) {
                double se = 0.0;
                int cnt = 0;
                bool pec = false;
                for (int u = -1; u <= 0; u++)
                    for (int v = -1; v <= 0; v++) {
                        int cc[3];
                        cc[c] = idx[c];
                        cc[c1] = idx[c1] + u;
                        cc[c2] = idx[c2] + v;
                        const int m = cell_id(p.n, p.per, p.px, p.id, cc[0], cc[1], cc[2]);
                        if (m < 0) continue;
                        se += p.mat[m].eps_r;
                        pec = pec || p.mat[m].is_pec;
                        cnt++;
                    }
                if (!pec && cnt) {
                    const double eps = p.eps0 * (se / cnt);
                    const double e = (double)p.E[c][q];
                    we += eps * e * e;
                }
            }
            double d1, d2;
            curl_e64(p, c, idx, d1, d2);
            const double cu = p.hcd * (d1 - d2);
            const double h = (double)p.H[c][q];
            wh += h * h - cu * cu;
        }
    }
    red[0][t] = we;
    red[1][t] = wh;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) {
            red[0][t] += red[0][t + s];
            red[1][t] += red[1][t + s];
        }
        __syncthreads();
    }
    if (t == 0) {
        const long long b = blockIdx.x + (long long)gridDim.x * (blockIdx.y + (long long)gridDim.y * blockIdx.z);
        part[2 * b] = red[0][0];
        part[2 * b + 1] = red[1][0];
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_zeeman(KParams<T> p) {
    __shared__ double red[256];
    const int4 bt = p.blocktab[blockIdx.x];
    const int f = bt.x, c = bt.y;
    const FilmDev &F = p.films[f];
    const long long l = (long long)bt.z + threadIdx.x;
    double z = 0.0;
    if (l < F.ns) {
        int idx[3];
        idx[0] = F.b0[0] + (int)(l % F.bn[0]);
        idx[1] = F.b0[1] + (int)((l / F.bn[0]) % F.bn[1]);
        idx[2] = F.b0[2] + (int)(l / ((long long)F.bn[0] * F.bn[1]));
        double ms, al, ga;
        site_params(p, c, idx, ms, al, ga);
        if (ms > 0.0) z = p.H0[c] * F.M[(c * 3 + c) * F.ns + l];
    }
    red[threadIdx.x] = z;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) p.partial[blockIdx.x] = red[0];
}

__global__ void k_sum_pairs(const double *part, long long n, double *out) {
    __shared__ double red[2][256];
    double a = 0.0, b = 0.0;
    for (long long t = threadIdx.x; t < n; t += blockDim.x) {
        a += part[2 * t];
        b += part[2 * t + 1];
    }
    red[0][threadIdx.x] = a;
    red[1][threadIdx.x] = b;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = red[0][0];
        out[1] = red[1][0];
    }
}

__global__ void k_sum(const double *part, long long n, double *out) {
    __shared__ double red[256];
    double a = 0.0;
    for (long long t = threadIdx.x; t < n; t += blockDim.x) a += part[t];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// ---------------------------------------------------------------------------
// host-side launchers (explicit instantiation for float and double)
// ---------------------------------------------------------------------------
template <typename T>
hipError_t launch_hbulk(const KParams<T> &p, int nhalf, int inc, hipStream_t s) {
    dim3 blk(64, 4, 1), grd((p.n[0] + 63) / 64, (p.n[1] + 3) / 4, p.n[2]);
    if (nhalf == 2)
        k_hbulk<T, 2><<<grd, blk, 0, s>>>(p, inc);
    else
        k_hbulk<T, 1><<<grd, blk, 0, s>>>(p, inc);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_epass(const KParams<T> &p, hipStream_t s) {
    dim3 blk(64, 4, 1), grd((p.n[0] + 63) / 64, (p.n[1] + 3) / 4, p.n[2]);
    hipLaunchKernelGGL(k_epass<T>, grd, blk, 0, s, p);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_film(const KParams<T> &p, int nblk, int phase, hipStream_t s) {
    if (nblk == 0) return hipSuccess;
    hipLaunchKernelGGL(k_film<T>, dim3(nblk), dim3(256), 0, s, p, phase);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_commit(const KParams<T> &p, int nblk, hipStream_t s) {
    if (nblk == 0) return hipSuccess;
    hipLaunchKernelGGL(k_film_commit<T>, dim3(nblk), dim3(256), 0, s, p);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_probes(const KParams<T> &p, int nprobe, hipStream_t s) {
    if (nprobe == 0) return hipSuccess;
    hipLaunchKernelGGL(k_probes<T>, dim3(nprobe), dim3(256), 0, s, p);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_energy(const KParams<T> &p, int nblk, double *part, double *out, hipStream_t s) {
    dim3 blk(64, 4, 1), grd((p.n[0] + 63) / 64, (p.n[1] + 3) / 4, p.n[2]);
    hipLaunchKernelGGL(k_energy<T>, grd, blk, 0, s, p, part);
    const long long nb = (long long)grd.x * grd.y * grd.z;
    hipLaunchKernelGGL(k_sum_pairs, dim3(1), dim3(256), 0, s, part, nb, out);
    if (nblk) {
        hipLaunchKernelGGL(k_zeeman<T>, dim3(nblk), dim3(256), 0, s, p);
        hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, p.partial, (long long)nblk, out + 2);
    }
    return hipGetLastError();
}

#define MPX_INSTANTIATE(T)                                                                  \
    template hipError_t launch_hbulk<T>(const KParams<T> &, int, int, hipStream_t);         \
    template hipError_t launch_epass<T>(const KParams<T> &, hipStream_t);                   \
    template hipError_t launch_film<T>(const KParams<T> &, int, int, hipStream_t);          \
    template hipError_t launch_commit<T>(const KParams<T> &, int, hipStream_t);             \
    template hipError_t launch_probes<T>(const KParams<T> &, int, hipStream_t);             \
    template hipError_t launch_energy<T>(const KParams<T> &, int, double *, double *, hipStream_t);

MPX_INSTANTIATE(float)
MPX_INSTANTIATE(double)

} // namespace mpx
