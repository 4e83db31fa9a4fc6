// adjoint.hip -- reverse-mode (discrete adjoint) kernels of the coupled step.
//
// The forward step (arXiv:2510.22221, Methods, "Numerical Model") is
//   HALF1(E^n): H/M half step (eq. iterate_H; LLG eqs. llg_tra4-llg_tra6 at
//               magnetic faces, solved in closed form and normalised),
//   ESTEP(H):   the E update after eq. iterate_H, with CPML and the source,
//   HALF2(E^{n+1}),
// and the adjoint runs the transposes of these maps in reverse order.  Given
// the adjoint state lambda of the state after a map and the map's input
// state (recomputed from checkpoints), a kernel here returns lambda of the
// input state and accumulates the parameter gradients:
//   * non-magnetic faces and E edges are linear: transposed curls and
//     transposed CPML recursions;
//   * a magnetic face's update M' = Ms X/|X|, X = (b + (a.b)a - a x b) /
//     (1 + |a|^2), a = -(k P + (alpha/Ms) M), b = M - k M x Q, with P, Q the
//     site's B^* and B^ (own component, and the mean of four neighbouring
//     faces of each other family) plus H0, is differentiated by hand; H0, Ms
//     of each face and the edge coefficients ca, cb collect gradients.
// One thread per slot or per film face; every sum a thread forms is a gather
// (no atomics), so results do not depend on scheduling.
#include "device_common.h"

namespace mpx {

__device__ __forceinline__ void cross3a(const double *a, const double *b, double *r) {
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ __forceinline__ double dot3a(const double *a, const double *b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// local index of face idx (folded) in the film's face box, -1 outside
__device__ __forceinline__ long long film_local_idx(const FilmDev &F, const int *idx) {
    const int r0 = idx[0] - F.b0[0], r1 = idx[1] - F.b0[1], r2 = idx[2] - F.b0[2];
    if (r0 < 0 || r0 >= F.bn[0] || r1 < 0 || r1 >= F.bn[1] || r2 < 0 || r2 >= F.bn[2]) return -1;
    return (long long)r0 + (long long)F.bn[0] * ((long long)r1 + (long long)F.bn[1] * r2);
}

// the magnetic face of family c at idx: (film, local index) or (-1, -1)
template <typename T>
__device__ __forceinline__ int mag_site(const KParams<T> &p, int c, const int *idx, long long &l) {
    for (int f = 0; f < p.nfilm; f++) {
        const FilmDev &F = p.films[f];
        const long long q = film_local_idx(F, idx);
        if (q >= 0) {
            if (F.prm[(c * 3) * F.ns + q] > 0.0) {
                l = q;
                return f;
            }
            return -1;
        }
    }
    l = -1;
    return -1;
}

// ---------------------------------------------------------------------------
// magnetic faces: lambda of (M', H'_c) -> lambda of M (direct), P, Q; the
// prepass (B^n, B^* of the input state) must have run
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_adj_film(AdjParams<T> A) {
    const KParams<T> &p = A.p;
    const int4 bt = block_entry(p.blocktab, blockIdx.x);
    const int f = bt.x, c = bt.y;
    const FilmDev F = film_desc(p.films, f);
    const AdjFilmDev G = scalar_desc(A.af, f);
    const long long l = (long long)bt.z + threadIdx.x;
    if (l >= F.ns) return;
    const double ms = F.prm[(c * 3 + 0) * F.ns + l];
    const double al = F.prm[(c * 3 + 1) * F.ns + l];
    const double ga = F.prm[(c * 3 + 2) * F.ns + l];
    if (!(ms > 0.0)) return;
    int idx[3];
    idx[0] = F.b0[0] + (int)(l % F.bn[0]);
    idx[1] = F.b0[1] + (int)((l / F.bn[0]) % F.bn[1]);
    idx[2] = F.b0[2] + (int)(l / ((long long)F.bn[0] * F.bn[1]));
    auto ext = [&](const int *q) -> long long {
        const int r0 = q[0] - F.e0[0], r1 = q[1] - F.e0[1], r2 = q[2] - F.e0[2];
        if (r0 < 0 || r0 >= F.en[0] || r1 < 0 || r1 >= F.en[1] || r2 < 0 || r2 >= F.en[2]) return -1;
        return (long long)r0 + (long long)F.en[0] * ((long long)r1 + (long long)F.en[1] * r2);
    };
    // the forward quantities (as the film kernel computes them)
    const long long le = ext(idx);
    double P[3], Q[3], M[3];
    P[c] = le >= 0 ? F.Bs[c * F.nse + le] : 0.0;
    Q[c] = le >= 0 ? F.Bn[c * F.nse + le] : 0.0;
    for (int cp = 0; cp < 3; cp++) {
        if (cp == c) continue;
        double vn[2][2], vs[2][2];
        for (int u = 0; u < 2; u++)
            for (int v = 0; v < 2; v++) {
                int q[3] = {idx[0], idx[1], idx[2]};
                q[c] += u - 1;
                q[cp] += v;
                for (int a = 0; a < 3; a++) q[a] = fold(q[a], p.n[a], p.per[a]);
                const long long lq = ext(q);
                vn[u][v] = lq >= 0 ? F.Bn[cp * F.nse + lq] : 0.0;
                vs[u][v] = lq >= 0 ? F.Bs[cp * F.nse + lq] : 0.0;
            }
        Q[cp] = ((vn[0][0] + vn[1][0]) + (vn[0][1] + vn[1][1])) * 0.25;
        P[cp] = ((vs[0][0] + vs[1][0]) + (vs[0][1] + vs[1][1])) * 0.25;
    }
    for (int w = 0; w < 3; w++) {
        P[w] += p.H0[w];
        Q[w] += p.H0[w];
        M[w] = F.M[(c * 3 + w) * F.ns + l];
    }
    const double kk = p.kf * ga;
    double MxQ[3], b[3], a[3];
    cross3a(M, Q, MxQ);
    for (int w = 0; w < 3; w++) b[w] = M[w] - kk * MxQ[w];
    for (int w = 0; w < 3; w++) a[w] = -(kk * P[w] + (al / ms) * M[w]);
    double axb[3], X[3];
    cross3a(a, b, axb);
    const double ab = dot3a(a, b), aa = dot3a(a, a);
    const double D = 1.0 + aa;
    for (int w = 0; w < 3; w++) X[w] = (b[w] + ab * a[w] - axb[w]) / D;
    const double nx = sqrt(dot3a(X, X));
    double u[3];
    for (int w = 0; w < 3; w++) u[w] = X[w] / nx;

    // lambda of M' (the face's H' = B^*_c - M'_c contributes -lambda H'_c)
    const long long sl = p.slot(idx[0], idx[1], idx[2]);
    double lMt[3];
    for (int w = 0; w < 3; w++) lMt[w] = G.lM[(c * 3 + w) * F.ns + l];
    lMt[c] -= (double)A.lH[c][sl];
    // M' = Ms u, u = X/|X|
    const double ul = dot3a(u, lMt);
    double gms = ul;
    double lX[3];
    for (int w = 0; w < 3; w++) lX[w] = ms * (lMt[w] - u[w] * ul) / nx;
    // X = N / D, N = b + (a.b) a - a x b, D = 1 + a.a
    double lN[3];
    for (int w = 0; w < 3; w++) lN[w] = lX[w] / D;
    const double lD = -dot3a(lX, X) / D;
    const double alN = dot3a(a, lN);
    double lNxb[3], lNxa[3];
    cross3a(lN, b, lNxb);
    cross3a(lN, a, lNxa);
    double la[3], lb[3];
    for (int w = 0; w < 3; w++) {
        la[w] = 2.0 * a[w] * lD + b[w] * alN + ab * lN[w] + lNxb[w];
        lb[w] = lN[w] + a[w] * alN - lNxa[w];
    }
    // a = -(k P + (alpha/Ms) M);  b = M - k M x Q
    double lP[3], lQ[3], lMd[3], Qxlb[3], lbxM[3];
    cross3a(Q, lb, Qxlb);
    cross3a(lb, M, lbxM);
    for (int w = 0; w < 3; w++) {
        lP[w] = -kk * la[w];
        lQ[w] = -kk * lbxM[w];
        lMd[w] = -(al / ms) * la[w] + lb[w] - kk * Qxlb[w];
    }
    gms += (al / (ms * ms)) * dot3a(M, la);
    for (int w = 0; w < 3; w++) {
        G.lp[(c * 3 + w) * F.ns + l] = lP[w];
        G.lq[(c * 3 + w) * F.ns + l] = lQ[w];
        G.lMout[(c * 3 + w) * F.ns + l] = lMd[w];
        G.gH0[(c * 3 + w) * F.ns + l] += lP[w] + lQ[w];
    }
    G.gMs[c * F.ns + l] += gms;
}

// can the face at idx be magnetic or be read by a magnetic face's solve (a
// face within one slot of a film's face box on every non-periodic axis)?
template <typename T>
__device__ __forceinline__ bool near_film(const KParams<T> &p, const int *idx) {
    for (int f = 0; f < p.nfilm; f++) {
        const FilmDev &F = p.films[f];
        bool in = true;
        for (int a = 0; a < 3; a++)
            if (!p.per[a] && (idx[a] < F.b0[a] - 1 || idx[a] > F.b0[a] + F.bn[a])) in = false;
        if (in) return true;
    }
    return false;
}

// ---------------------------------------------------------------------------
// every face: lambda of H' (and psi') -> lambda of H (and psi), the face's
// curl-part adjoints aD, and for magnetic faces lambda of M from B^
// ---------------------------------------------------------------------------
// lin1/lin2: lambda psiH of the derivative axes C+1, C+2 before the map;
// lout1/lout2: where the values after it go (the same arrays in place)
template <typename T, int C>
__device__ __forceinline__ void adj_face_core(const AdjParams<T> &A, const int *idx, const T *lin1, const T *lin2,
                                              T *lout1, T *lout2, T &ad0, T &ad1) {
    constexpr int C1 = (C + 1) % 3, C2 = (C + 2) % 3;
    const KParams<T> &p = A.p;
    const int i = idx[0], j = idx[1], k = idx[2];
    const long long q = p.slot(i, j, k);
    const T lHp = A.lH[C][q];
    const int a1 = idx[C1], a2 = idx[C2];
    const bool s1 = p.psiH[C][C1] && (a1 < p.nlo[C1] || a1 >= p.n[C1] - p.nhi[C1]);
    const bool s2 = p.psiH[C][C2] && (a2 < p.nlo[C2] || a2 >= p.n[C2] - p.nhi[C2]);
    const bool film_reach = p.nfilm && near_film(p, idx);
    if (!film_reach && !s1 && !s2) {
        // bulk face out of every film's reach: H' = H - hc (d1 - d2)
        ad0 = -(p.hc * lHp);
        ad1 = p.hc * lHp;
        return; // lambda H unchanged
    }
    long long lm;
    const int fm = film_reach ? mag_site(p, C, idx, lm) : -1;
    // CPML face (never next to a film)
    if (fm < 0 && (s1 || s2)) {
        const T g1 = -p.hc * lHp, g2 = p.hc * lHp; // d H' / d (d1 + psi1'), d (d2 + psi2')
        ad0 = g1;
        ad1 = g2;
        if (s1) {
            const long long qq = p.psi_index(C1, idx);
            const T aps = lin1[qq] + g1;
            lout1[qq] = p.bH[C1][a1] * aps;
            ad0 = g1 + p.cH[C1][a1] * aps;
        }
        if (s2) {
            const long long qq = p.psi_index(C2, idx);
            const T aps = lin2[qq] + g2;
            lout2[qq] = p.bH[C2][a2] * aps;
            ad1 = g2 + p.cH[C2][a2] * aps;
        }
        return; // lambda H unchanged (dH'/dH = 1)
    }
    // lambda of B^* and B^ of this face: from the face's own update and from
    // the solves of magnetic faces that read it (P, Q of the film kernel)
    double lbs_f = 0.0, lbn = 0.0;
    if (fm >= 0) {
        const FilmDev &F = p.films[fm];
        const AdjFilmDev &G = A.af[fm];
        lbs_f += G.lp[(C * 3 + C) * F.ns + lm];
        lbn += G.lq[(C * 3 + C) * F.ns + lm];
    }
    // transverse reads: the magnetic faces s of each other family cs with this
    // face in their four-face mean: s = t + a e_cs - b e_C, a, b in {0, 1}
    if (film_reach) {
#pragma unroll
        for (int cs = 0; cs < 3; cs++) {
            if (cs == C) continue;
            for (int aa = 0; aa < 2; aa++)
                for (int bb = 0; bb < 2; bb++) {
                    int s[3] = {i, j, k};
                    s[cs] += aa;
                    s[C] -= bb;
                    bool ok = true;
                    for (int ax = 0; ax < 3; ax++) {
                        s[ax] = fold(s[ax], p.n[ax], p.per[ax]);
                        if (s[ax] < 0) ok = false;
                    }
                    if (!ok) continue;
                    long long ls;
                    const int fs = mag_site(p, cs, s, ls);
                    if (fs < 0) continue;
                    const FilmDev &F = p.films[fs];
                    const AdjFilmDev &G = A.af[fs];
                    lbs_f += 0.25 * G.lp[(cs * 3 + C) * F.ns + ls];
                    lbn += 0.25 * G.lq[(cs * 3 + C) * F.ns + ls];
                }
        }
    }
    if (fm >= 0) {
        // magnetic face: H' = B^*_C - M'_C, B^* = B^ - hc (d1 - d2) in float64,
        // B^ = H + M_C
        const double lbs = (double)lHp + lbs_f;
        const double lbt = lbn + lbs;
        A.lH[C][q] = (T)lbt;
        const FilmDev &F = p.films[fm];
        const AdjFilmDev &G = A.af[fm];
        G.lMout[(C * 3 + C) * F.ns + lm] += lbt;
        ad0 = (T)(-p.hcd * lbs);
        ad1 = (T)(p.hcd * lbs);
    } else {
        // bulk face: H' = H - hc (d1 - d2) in the field precision; its B^ and
        // B^* as read by the solves are H and H - hc (d1 - d2) in float64
        A.lH[C][q] = (T)((double)lHp + lbn + lbs_f);
        ad0 = (T)(-(double)p.hc * (double)lHp - p.hcd * lbs_f);
        ad1 = (T)((double)p.hc * (double)lHp + p.hcd * lbs_f);
    }
}

template <typename T, int C>
__device__ __forceinline__ void adj_face(const AdjParams<T> &A, int i, int j, int k) {
    constexpr int C1 = (C + 1) % 3, C2 = (C + 2) % 3;
    const int idx[3] = {i, j, k};
    T a0, a1;
    adj_face_core<T, C>(A, idx, A.lpsiH[C][C1], A.lpsiH[C][C2], A.lpsiH[C][C1], A.lpsiH[C][C2], a0, a1);
    const long long q = A.p.slot(i, j, k);
    A.aD[C][0][q] = a0;
    A.aD[C][1][q] = a1;
}


template <typename T>
__global__ void __launch_bounds__(256) k_adj_face(AdjParams<T> A) {
    const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y, k = blockIdx.z;
    if (i >= A.p.n[0] || j >= A.p.n[1]) return;
    adj_face<T, 0>(A, i, j, k);
    adj_face<T, 1>(A, i, j, k);
    adj_face<T, 2>(A, i, j, k);
}

// magnetic faces: lambda of M before the map (the face kernel has added the
// B^ part); copies lMout -> lM
__global__ void __launch_bounds__(256) k_adj_film_commit(const int4 *blocktab, const FilmDev *films,
                                                         const AdjFilmDev *af) {
    const int4 bt = blocktab[blockIdx.x];
    const FilmDev &F = films[bt.x];
    const AdjFilmDev &G = af[bt.x];
    const int c = bt.y;
    const long long l = (long long)bt.z + threadIdx.x;
    if (l >= F.ns || !(F.prm[(c * 3) * F.ns + l] > 0.0)) return;
    for (int w = 0; w < 3; w++) G.lM[(c * 3 + w) * F.ns + l] = G.lMout[(c * 3 + w) * F.ns + l];
}

// face adjoints of a slot (folded; zero outside)
template <typename T>
__device__ __forceinline__ T ldD(const KParams<T> &p, const T *a, int i, int j, int k) {
    return ldz(p, a, i, j, k);
}

// lambda E += (transposed curl of E) applied to the faces' aD
template <typename T, int C>
__device__ __forceinline__ void adj_curlE(const AdjParams<T> &A, int i, int j, int k) {
    constexpr int C1 = (C + 1) % 3, C2 = (C + 2) % 3;
    const KParams<T> &p = A.p;
    // family C+1 (= C1): E_C enters its d1 along C2 ; family C+2 (= C2): its d2 along C1
    int u1[3] = {i, j, k}, u2[3] = {i, j, k};
    u1[C2] -= 1;
    u2[C1] -= 1;
    const T a1 = ldD(p, A.aD[C1][0], u1[0], u1[1], u1[2]) - ldD(p, A.aD[C1][0], i, j, k);
    const T a2 = ldD(p, A.aD[C2][1], u2[0], u2[1], u2[2]) - ldD(p, A.aD[C2][1], i, j, k);
    const long long q = p.slot(i, j, k);
    A.lE[C][q] = A.lE[C][q] + (dif(a1, T(0), p.dT[C2], p.invd[C2]) + dif(a2, T(0), p.dT[C1], p.invd[C1]));
}

template <typename T>
__global__ void __launch_bounds__(256) k_adj_curlE(AdjParams<T> A) {
    const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y, k = blockIdx.z;
    if (i >= A.p.n[0] || j >= A.p.n[1]) return;
    adj_curlE<T, 0>(A, i, j, k);
    adj_curlE<T, 1>(A, i, j, k);
    adj_curlE<T, 2>(A, i, j, k);
}

// ---------------------------------------------------------------------------
// E step: lambda E' (and psi') -> lambda E (and psi), the edge's curl-part
// adjoints eD, and dL/dca, dL/dcb
// ---------------------------------------------------------------------------
template <typename T, int C>
__device__ __forceinline__ void adj_edge(const AdjParams<T> &A, int i, int j, int k, long long step) {
    constexpr int C1 = (C + 1) % 3, C2 = (C + 2) % 3;
    const KParams<T> &p = A.p;
    const long long q = p.slot(i, j, k);
    int idx[3] = {i, j, k};
    // coefficients (zero for a PEC or wall edge: E' = 0 does not depend on anything)
    bool valid = true;
    for (int a = 0; a < 3; a++)
        if (!p.per[a] && a != C && idx[a] == 0) valid = false;
    double ca = 0.0, cb = 0.0;
    if (valid) {
        int m[4];
        for (int u = 0; u < 2; u++)
            for (int v = 0; v < 2; v++) {
                int cc[3] = {i, j, k};
                cc[C1] -= 1 - u;
                cc[C2] -= 1 - v;
                for (int a = 0; a < 3; a++) cc[a] = fold(cc[a], p.n[a], p.per[a]);
                m[2 * u + v] = p.id[p.slot(cc[0], cc[1], cc[2])];
            }
        const MatDev &M0 = p.mat[m[0]], &M1 = p.mat[m[1]], &M2 = p.mat[m[2]], &M3 = p.mat[m[3]];
        if (M0.is_pec || M1.is_pec || M2.is_pec || M3.is_pec) {
            valid = false;
        } else {
            double se = 0.0, ss = 0.0;
            se += M0.eps_r;
            ss += M0.sigma;
            se += M1.eps_r;
            ss += M1.sigma;
            se += M2.eps_r;
            ss += M2.sigma;
            se += M3.eps_r;
            ss += M3.sigma;
            const double eps = p.eps0 * (se / 4), sig = ss / 4;
            const double den = sig / 2.0 + eps / p.dt;
            ca = -(sig / 2.0 - eps / p.dt) / den;
            cb = 1.0 / den;
        }
    }
    if (!valid) {
        A.lE[C][q] = T(0);
        A.eD[C][0][q] = T(0);
        A.eD[C][1][q] = T(0);
        return;
    }
    // forward quantities: raw curl parts of H, psi', the source
    int d1i[3] = {i, j, k}, d2i[3] = {i, j, k};
    d1i[C1] -= 1;
    d2i[C2] -= 1;
    T d1 = dif(ldz(p, p.H[C2], i, j, k), ldz(p, p.H[C2], d1i[0], d1i[1], d1i[2]), p.dT[C1], p.invd[C1]);
    T d2 = dif(ldz(p, p.H[C1], i, j, k), ldz(p, p.H[C1], d2i[0], d2i[1], d2i[2]), p.dT[C2], p.invd[C2]);
    const int a1 = idx[C1], a2 = idx[C2];
    const bool s1 = p.psiE[C][C1] && (a1 < p.nlo[C1] || a1 >= p.n[C1] - p.nhi[C1]);
    const bool s2 = p.psiE[C][C2] && (a2 < p.nlo[C2] || a2 >= p.n[C2] - p.nhi[C2]);
    long long q1 = 0, q2 = 0;
    T b1 = T(0), c1 = T(0), b2 = T(0), c2 = T(0);
    if (s1) {
        q1 = p.psi_index(C1, idx);
        b1 = p.bE[C1][a1];
        c1 = p.cE[C1][a1];
        d1 += b1 * p.psiE[C][C1][q1] + c1 * d1;
    }
    if (s2) {
        q2 = p.psi_index(C2, idx);
        b2 = p.bE[C2][a2];
        c2 = p.cE[C2][a2];
        d2 += b2 * p.psiE[C][C2][q2] + c2 * d2;
    }
    double J = 0.0;
    for (int s = 0; s < p.nsrc; s++) {
        const SrcDev &S = p.srcs[s];
        if (S.comp != C) continue;
        if (idx[0] < S.box[0] || idx[0] >= S.box[0] + S.box[3] || idx[1] < S.box[1] || idx[1] >= S.box[1] + S.box[4] ||
            idx[2] < S.box[2] || idx[2] >= S.box[2] + S.box[5])
            continue;
        if (step < S.n) J += S.table[step];
    }
    const double x = (double)(d1 - d2) - J;
    const T lEp = A.lE[C][q];
    A.gca[C][q] += (double)lEp * (double)p.E[C][q];
    A.gcb[C][q] += (double)lEp * x;
    const T lx = (T)cb * lEp;
    A.lE[C][q] = (T)ca * lEp;
    // x = (d1 + psi1') - (d2 + psi2') - J, psi' = b psi + c d
    T ad1 = lx, ad2 = -lx;
    if (s1) {
        const T aps = A.lpsiE[C][C1][q1] + lx;
        A.lpsiE[C][C1][q1] = b1 * aps;
        ad1 = lx + c1 * aps;
    }
    if (s2) {
        const T aps = A.lpsiE[C][C2][q2] - lx;
        A.lpsiE[C][C2][q2] = b2 * aps;
        ad2 = -lx + c2 * aps;
    }
    A.eD[C][0][q] = ad1;
    A.eD[C][1][q] = ad2;
}

template <typename T>
__global__ void __launch_bounds__(256) k_adj_estep(AdjParams<T> A) {
    const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y, k = blockIdx.z;
    if (i >= A.p.n[0] || j >= A.p.n[1]) return;
    const long long step = A.p.step[0];
    adj_edge<T, 0>(A, i, j, k, step);
    adj_edge<T, 1>(A, i, j, k, step);
    adj_edge<T, 2>(A, i, j, k, step);
}

// lambda H += (transposed curl of H) applied to the edges' eD
template <typename T, int C>
__device__ __forceinline__ void adj_curlH(const AdjParams<T> &A, int i, int j, int k) {
    constexpr int C1 = (C + 1) % 3, C2 = (C + 2) % 3;
    const KParams<T> &p = A.p;
    // H_C is the H_{C2} of edges E_{C1} (their d1, along C2) and the H_{C1} of
    // edges E_{C2} (their d2, along C1)
    int u1[3] = {i, j, k}, u2[3] = {i, j, k};
    u1[C2] += 1;
    u2[C1] += 1;
    const T a1 = ldz(p, A.eD[C1][0], i, j, k) - ldz(p, A.eD[C1][0], u1[0], u1[1], u1[2]);
    const T a2 = ldz(p, A.eD[C2][1], i, j, k) - ldz(p, A.eD[C2][1], u2[0], u2[1], u2[2]);
    const long long q = p.slot(i, j, k);
    A.lH[C][q] = A.lH[C][q] + (dif(a1, T(0), p.dT[C2], p.invd[C2]) + dif(a2, T(0), p.dT[C1], p.invd[C1]));
}

template <typename T>
__global__ void __launch_bounds__(256) k_adj_curlH(AdjParams<T> A) {
    const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y, k = blockIdx.z;
    if (i >= A.p.n[0] || j >= A.p.n[1]) return;
    adj_curlH<T, 0>(A, i, j, k);
    adj_curlH<T, 1>(A, i, j, k);
    adj_curlH<T, 2>(A, i, j, k);
}

// ---------------------------------------------------------------------------
// the loss: scale * (film EM energy of film f) of the current state -> its
// gradient added to lambda E, lambda H
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ bool film_cell(const KParams<T> &p, const FilmDev &F, int i, int j, int k, double &eps) {
    if (i < F.cb[0] || i >= F.cb[0] + F.cb[3] || j < F.cb[1] || j >= F.cb[1] + F.cb[4] || k < F.cb[2] ||
        k >= F.cb[2] + F.cb[5])
        return false;
    const MatDev &m = p.mat[p.id[p.slot(i, j, k)]];
    eps = m.eps_r;
    return m.Ms > 0.0;
}

template <typename T>
__global__ void __launch_bounds__(256) k_adj_loss(AdjParams<T> A, int film, double scale) {
    const KParams<T> &p = A.p;
    const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y, k = blockIdx.z;
    if (i >= p.n[0] || j >= p.n[1]) return;
    const FilmDev &F = p.films[film];
    const long long q = p.slot(i, j, k);
    for (int C = 0; C < 3; C++) {
        const int C1 = (C + 1) % 3, C2 = (C + 2) % 3;
        // E_C at the slot: the cells at (C1, C2) offsets -1 / 0
        double se = 0.0;
        for (int u = 0; u < 2; u++)
            for (int v = 0; v < 2; v++) {
                int cc[3] = {i, j, k};
                cc[C1] -= u;
                cc[C2] -= v;
                double eps;
                if (film_cell(p, F, cc[0], cc[1], cc[2], eps)) se += eps;
            }
        if (se != 0.0) A.lE[C][q] += (T)(scale * p.dV * p.eps0 * se * 0.25 * (double)p.E[C][q]);
        // H_C at the slot: the cells at C offsets -1 / 0
        int nc = 0;
        for (int u = 0; u < 2; u++) {
            int cc[3] = {i, j, k};
            cc[C] -= u;
            double eps;
            if (film_cell(p, F, cc[0], cc[1], cc[2], eps)) nc++;
        }
        if (nc) A.lH[C][q] += (T)(scale * p.dV * p.mu0 * 0.5 * nc * (double)p.H[C][q]);
    }
}

// lambda M of the initial magnetisation M0 = Ms u at every magnetic face ->
// dL/dMs of the face
__global__ void __launch_bounds__(256) k_adj_init_ms(const int4 *blocktab, const FilmDev *films,
                                                     const AdjFilmDev *af, double u0, double u1, double u2) {
    const int4 bt = blocktab[blockIdx.x];
    const FilmDev &F = films[bt.x];
    const AdjFilmDev &G = af[bt.x];
    const int c = bt.y;
    const long long l = (long long)bt.z + threadIdx.x;
    if (l >= F.ns || !(F.prm[(c * 3) * F.ns + l] > 0.0)) return;
    G.gMs[c * F.ns + l] += G.lM[(c * 3 + 0) * F.ns + l] * u0 + G.lM[(c * 3 + 1) * F.ns + l] * u1 +
                           G.lM[(c * 3 + 2) * F.ns + l] * u2;
}

// dL/d eps_r of the cells of a box from the accumulated dL/dca, dL/dcb of
// the twelve edges around each cell (eps of an edge: eps0 x the mean over
// its four cells)
template <typename T>
__global__ void __launch_bounds__(256) k_adj_eps(AdjParams<T> A, int4 b0, int4 bn, double *out) {
    const KParams<T> &p = A.p;
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long ncell = (long long)bn.x * bn.y * bn.z;
    if (t >= ncell) return;
    const int ci = b0.x + (int)(t % bn.x), cj = b0.y + (int)((t / bn.x) % bn.y), ck = b0.z + (int)(t / ((long long)bn.x * bn.y));
    double g = 0.0;
    for (int C = 0; C < 3; C++) {
        const int C1 = (C + 1) % 3, C2 = (C + 2) % 3;
        for (int u = 0; u < 2; u++)
            for (int v = 0; v < 2; v++) {
                int e[3] = {ci, cj, ck};
                e[C1] += u;
                e[C2] += v;
                for (int a = 0; a < 3; a++) e[a] = fold(e[a], p.n[a], p.per[a]);
                if (e[0] < 0 || e[1] < 0 || e[2] < 0) continue;
                bool valid = true;
                for (int a = 0; a < 3; a++)
                    if (!p.per[a] && a != C && e[a] == 0) valid = false;
                if (!valid) continue;
                int m[4];
                for (int uu = 0; uu < 2; uu++)
                    for (int vv = 0; vv < 2; vv++) {
                        int cc[3] = {e[0], e[1], e[2]};
                        cc[C1] -= 1 - uu;
                        cc[C2] -= 1 - vv;
                        for (int a = 0; a < 3; a++) cc[a] = fold(cc[a], p.n[a], p.per[a]);
                        m[2 * uu + vv] = p.id[p.slot(cc[0], cc[1], cc[2])];
                    }
                const MatDev &M0 = p.mat[m[0]], &M1 = p.mat[m[1]], &M2 = p.mat[m[2]], &M3 = p.mat[m[3]];
                if (M0.is_pec || M1.is_pec || M2.is_pec || M3.is_pec) continue;
                const double eps = p.eps0 * ((M0.eps_r + M1.eps_r + M2.eps_r + M3.eps_r) / 4);
                const double sig = (M0.sigma + M1.sigma + M2.sigma + M3.sigma) / 4;
                const double den = sig / 2.0 + eps / p.dt;
                // ca = (eps/dt - sig/2)/den, cb = 1/den
                const double dca = (sig / p.dt) / (den * den), dcb = -(1.0 / p.dt) / (den * den);
                const long long q = p.slot(e[0], e[1], e[2]);
                g += (A.gca[C][q] * dca + A.gcb[C][q] * dcb) * (p.eps0 / 4.0);
            }
    }
    out[t] = g;
}

// the film EM energy of film f in the current state (the film-energy probe's
// sum): per-block partials, summed on the host in block order
template <typename T>
__global__ void __launch_bounds__(256) k_film_energy(KParams<T> p, int film, double *part) {
    __shared__ double red[256];
    const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y, k = blockIdx.z;
    const int tid = threadIdx.y * 64 + threadIdx.x;
    double w = 0.0;
    const FilmDev &F = p.films[film];
    double eps;
    if (i < p.n[0] && j < p.n[1] && film_cell(p, F, i, j, k, eps)) {
        const int cc[3] = {i, j, k};
        double we = 0.0, wh = 0.0;
        for (int c = 0; c < 3; c++) {
            const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
            double e2 = 0.0;
            for (int u = 0; u < 2; u++)
                for (int v = 0; v < 2; v++) {
                    int q[3] = {cc[0], cc[1], cc[2]};
                    q[c1] += u;
                    q[c2] += v;
                    const double e = (double)ldz(p, p.E[c], q[0], q[1], q[2]);
                    e2 += e * e;
                }
            we += e2 / 4.0;
            double h2 = 0.0;
            for (int u = 0; u < 2; u++) {
                int q[3] = {cc[0], cc[1], cc[2]};
                q[c] += u;
                const double h = (double)ldz(p, p.H[c], q[0], q[1], q[2]);
                h2 += h * h;
            }
            wh += h2 / 2.0;
        }
        w = (0.5 * p.eps0 * eps * we + 0.5 * p.mu0 * wh) * p.dV;
    }
    red[tid] = w;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (tid < st) red[tid] += red[tid + st];
        __syncthreads();
    }
    if (tid == 0) part[blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)] = red[0];
}

__global__ void k_set_step(long long *step, long long v) {
    if (threadIdx.x == 0) step[0] = v;
}

// acc += scale * (sum of the partials in order), one thread: deterministic
__global__ void k_accum(const double *part, int n, double *acc, double scale) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int q = 0; q < n; q++) s += part[q];
    acc[0] += scale * s;
}

// ---------------------------------------------------------------------------
// tape schedule
// ---------------------------------------------------------------------------

// A region of slots [b0, b0 + r) (a cell box grown by one slot on the high
// side of each axis: the edges and faces of its cells).  Thread t owns the
// slot of region index t after folding; a slot that the fold maps onto an
// index the region already holds (a box spanning a periodic axis) belongs to
// that index.  Returns false for no slot or a slot owned elsewhere.
__device__ __forceinline__ bool region_slot(const int *n, const int *per, const int *b0, const int *r, long long t,
                                            int *q) {
    const int loc[3] = {(int)(t % r[0]), (int)((t / r[0]) % r[1]), (int)(t / ((long long)r[0] * r[1]))};
    for (int a = 0; a < 3; a++) {
        int v = b0[a] + loc[a];
        if (v >= n[a]) {
            if (!per[a]) return false;
            v -= n[a];
            if (v >= b0[a]) return false;
        }
        q[a] = v;
    }
    return true;
}

// region index of the slot e (unfolded, inside [b0, b0 + r) or its wrap), -1
// for no slot
__device__ __forceinline__ long long region_index(const int *n, const int *per, const int *b0, const int *r,
                                                  const int *e) {
    int loc[3];
    for (int a = 0; a < 3; a++) {
        int v = e[a];
        if (v >= n[a]) {
            if (!per[a]) return -1;
            if (v - n[a] >= b0[a]) v -= n[a];
        }
        loc[a] = v - b0[a];
        if (loc[a] < 0 || loc[a] >= r[a]) return -1;
    }
    return (long long)loc[0] + (long long)r[0] * ((long long)loc[1] + (long long)r[1] * loc[2]);
}

// the film's E and H at an integer time over its cell box grown by one slot:
// [6][region] (Ex, Ey, Ez, Hx, Hy, Hz).  merged = 1: between the two film half
// steps of a merged pair (magnetic faces' H in the film's staging, bulk faces'
// H one bulk half step ahead of the stored H); 0: a state at an integer time
template <typename T>
__global__ void __launch_bounds__(256) k_tape_loss(KParams<T> p, int film, int merged, double *dst) {
    const FilmDev &F = p.films[film];
    const int b0[3] = {F.cb[0], F.cb[1], F.cb[2]}, r[3] = {F.cb[3] + 1, F.cb[4] + 1, F.cb[5] + 1};
    const long long tb = (long long)r[0] * r[1] * r[2];
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= tb) return;
    int q[3];
    if (!region_slot(p.n, p.per, b0, r, t, q)) {
        for (int w = 0; w < 6; w++) dst[w * tb + t] = 0.0;
        return;
    }
    const long long sl = p.slot(q[0], q[1], q[2]);
    for (int C = 0; C < 3; C++) {
        dst[C * tb + t] = (double)p.E[C][sl];
        double h;
        long long l;
        const int f = merged && p.nfilm ? mag_site(p, C, q, l) : -1;
        if (!merged) {
            h = (double)p.H[C][sl];
        } else if (f >= 0) {
            h = p.films[f].H1[C * p.films[f].ns + l];
        } else {
            const int C1 = (C + 1) % 3, C2 = (C + 2) % 3;
            int u1[3] = {q[0], q[1], q[2]}, u2[3] = {q[0], q[1], q[2]};
            u1[C1] += 1;
            u2[C2] += 1;
            const T d1 = dif(ldz(p, p.E[C2], u1[0], u1[1], u1[2]), p.E[C2][sl], p.dT[C1], p.invd[C1]);
            const T d2 = dif(ldz(p, p.E[C1], u2[0], u2[1], u2[2]), p.E[C1][sl], p.dT[C2], p.invd[C2]);
            h = (double)(p.H[C][sl] - p.hc * (d1 - d2));
        }
        dst[(3 + C) * tb + t] = h;
    }
}

// the loss term of the state a tape slot holds: scale x the gradient of the
// film EM energy added to lambda E and lambda H; no-op unless the slot's
// time index seg0 + m is past loss_from (seg0 null: always)
template <typename T>
__global__ void __launch_bounds__(256) k_adj_loss_tape(AdjParams<T> A, int film, double scale, const double *tape,
                                                       const long long *seg0, int m, long long loss_from) {
    if (seg0 && seg0[0] + m <= loss_from) return;
    const KParams<T> &p = A.p;
    const FilmDev &F = p.films[film];
    const int b0[3] = {F.cb[0], F.cb[1], F.cb[2]}, r[3] = {F.cb[3] + 1, F.cb[4] + 1, F.cb[5] + 1};
    const long long tb = (long long)r[0] * r[1] * r[2];
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    int q[3];
    if (t >= tb || !region_slot(p.n, p.per, b0, r, t, q)) return;
    const long long sl = p.slot(q[0], q[1], q[2]);
    for (int C = 0; C < 3; C++) {
        const int C1 = (C + 1) % 3, C2 = (C + 2) % 3;
        double se = 0.0, eps;
        for (int u = 0; u < 2; u++)
            for (int v = 0; v < 2; v++) {
                int cc[3] = {q[0], q[1], q[2]};
                cc[C1] -= u;
                cc[C2] -= v;
                for (int a = 0; a < 3; a++) cc[a] = fold(cc[a], p.n[a], p.per[a]);
                if (cc[0] >= 0 && cc[1] >= 0 && cc[2] >= 0 && film_cell(p, F, cc[0], cc[1], cc[2], eps)) se += eps;
            }
        if (se != 0.0) A.lE[C][sl] += (T)(scale * p.dV * p.eps0 * se * 0.25 * tape[C * tb + t]);
        int nc = 0;
        for (int u = 0; u < 2; u++) {
            int cc[3] = {q[0], q[1], q[2]};
            cc[C] -= u;
            for (int a = 0; a < 3; a++) cc[a] = fold(cc[a], p.n[a], p.per[a]);
            if (cc[0] >= 0 && cc[1] >= 0 && cc[2] >= 0 && film_cell(p, F, cc[0], cc[1], cc[2], eps)) nc++;
        }
        if (nc) A.lH[C][sl] += (T)(scale * p.dV * p.mu0 * 0.5 * nc * tape[(3 + C) * tb + t]);
    }
}

// The loss's own dependence on eps_r: the film energy holds
// 1/2 eps0 eps_r dV times the mean over its four edges of E_C^2 (summed over
// C) for each film cell, so dL/d eps_r of a film cell collects that sum of
// every state in the loss window, x scale.  acc is [film cell box] (x
// fastest).  From a film-region tape slot (seg0 null: always; else only when
// seg0 + m is past loss_from) ...
template <typename T>
__global__ void __launch_bounds__(256) k_adj_loss_eps_tape(KParams<T> p, int film, double scale, const double *tape,
                                                           const long long *seg0, int m, long long loss_from,
                                                           double *acc) {
    if (seg0 && seg0[0] + m <= loss_from) return;
    const FilmDev &F = p.films[film];
    const int b0[3] = {F.cb[0], F.cb[1], F.cb[2]}, r[3] = {F.cb[3] + 1, F.cb[4] + 1, F.cb[5] + 1};
    const long long tb = (long long)r[0] * r[1] * r[2];
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long long)F.cb[3] * F.cb[4] * F.cb[5]) return;
    const int cell[3] = {F.cb[0] + (int)(t % F.cb[3]), F.cb[1] + (int)((t / F.cb[3]) % F.cb[4]),
                         F.cb[2] + (int)(t / ((long long)F.cb[3] * F.cb[4]))};
    double eps;
    if (!film_cell(p, F, cell[0], cell[1], cell[2], eps)) return;
    double we = 0.0;
    for (int C = 0; C < 3; C++) {
        const int C1 = (C + 1) % 3, C2 = (C + 2) % 3;
        double e2 = 0.0;
        for (int u = 0; u < 2; u++)
            for (int v = 0; v < 2; v++) {
                int e[3] = {cell[0], cell[1], cell[2]};
                e[C1] += u;
                e[C2] += v;
                const long long ri = region_index(p.n, p.per, b0, r, e);
                if (ri < 0) continue; // a wall edge: E = 0
                const double x = tape[C * tb + ri];
                e2 += x * x;
            }
        we += e2 / 4.0;
    }
    acc[t] += scale * 0.5 * p.eps0 * p.dV * we;
}

// ... or from the current state (the plain schedule)
template <typename T>
__global__ void __launch_bounds__(256) k_adj_loss_eps_state(KParams<T> p, int film, double scale, double *acc) {
    const FilmDev &F = p.films[film];
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long long)F.cb[3] * F.cb[4] * F.cb[5]) return;
    const int cell[3] = {F.cb[0] + (int)(t % F.cb[3]), F.cb[1] + (int)((t / F.cb[3]) % F.cb[4]),
                         F.cb[2] + (int)(t / ((long long)F.cb[3] * F.cb[4]))};
    double eps;
    if (!film_cell(p, F, cell[0], cell[1], cell[2], eps)) return;
    double we = 0.0;
    for (int C = 0; C < 3; C++) {
        const int C1 = (C + 1) % 3, C2 = (C + 2) % 3;
        double e2 = 0.0;
        for (int u = 0; u < 2; u++)
            for (int v = 0; v < 2; v++) {
                int q[3] = {cell[0], cell[1], cell[2]};
                q[C1] += u;
                q[C2] += v;
                const double x = (double)ldz(p, p.E[C], q[0], q[1], q[2]);
                e2 += x * x;
            }
        we += e2 / 4.0;
    }
    acc[t] += scale * 0.5 * p.eps0 * p.dV * we;
}

// E^n and x^n = (d1 + psi1') - (d2 + psi2') - J^n (the E update's input, H at
// n + 1/2) over the edges of a cell box: [6][region] (E0..2, x0..2); taken
// just before the E pass
template <typename T>
__global__ void __launch_bounds__(256) k_tape_box(KParams<T> p, int4 bb, int4 bs, double *dst) {
    const int b0[3] = {bb.x, bb.y, bb.z}, r[3] = {bs.x + 1, bs.y + 1, bs.z + 1};
    const long long tb = (long long)r[0] * r[1] * r[2];
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= tb) return;
    int q[3];
    if (!region_slot(p.n, p.per, b0, r, t, q)) {
        for (int w = 0; w < 6; w++) dst[w * tb + t] = 0.0;
        return;
    }
    const long long sl = p.slot(q[0], q[1], q[2]);
    const long long step = p.step[0];
    for (int C = 0; C < 3; C++) {
        const int C1 = (C + 1) % 3, C2 = (C + 2) % 3;
        int d1i[3] = {q[0], q[1], q[2]}, d2i[3] = {q[0], q[1], q[2]};
        d1i[C1] -= 1;
        d2i[C2] -= 1;
        T d1 = dif(p.H[C2][sl], ldz(p, p.H[C2], d1i[0], d1i[1], d1i[2]), p.dT[C1], p.invd[C1]);
        T d2 = dif(p.H[C1][sl], ldz(p, p.H[C1], d2i[0], d2i[1], d2i[2]), p.dT[C2], p.invd[C2]);
        const int a1 = q[C1], a2 = q[C2];
        if (p.psiE[C][C1] && (a1 < p.nlo[C1] || a1 >= p.n[C1] - p.nhi[C1]))
            d1 += p.bE[C1][a1] * p.psiE[C][C1][p.psi_index(C1, q)] + p.cE[C1][a1] * d1;
        if (p.psiE[C][C2] && (a2 < p.nlo[C2] || a2 >= p.n[C2] - p.nhi[C2]))
            d2 += p.bE[C2][a2] * p.psiE[C][C2][p.psi_index(C2, q)] + p.cE[C2][a2] * d2;
        double J = 0.0;
        for (int s = 0; s < p.nsrc; s++) {
            const SrcDev &S = p.srcs[s];
            if (S.comp != C) continue;
            if (q[0] < S.box[0] || q[0] >= S.box[0] + S.box[3] || q[1] < S.box[1] || q[1] >= S.box[1] + S.box[4] ||
                q[2] < S.box[2] || q[2] >= S.box[2] + S.box[5])
                continue;
            if (step < S.n) J += S.table[step];
        }
        dst[C * tb + t] = (double)p.E[C][sl];
        dst[(3 + C) * tb + t] = (double)(d1 - d2) - J;
    }
}

// dL/d eps_r of the box's cells from the box accumulators (eps of an edge:
// eps0 x the mean over its four cells)
template <typename T>
__global__ void __launch_bounds__(256) k_adj_eps_box(KParams<T> p, int4 bb, int4 bs, const double *gca,
                                                     const double *gcb, double *out) {
    const int b0[3] = {bb.x, bb.y, bb.z}, r[3] = {bs.x + 1, bs.y + 1, bs.z + 1};
    const long long tb = (long long)r[0] * r[1] * r[2];
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long ncell = (long long)bs.x * bs.y * bs.z;
    if (t >= ncell) return;
    const int cell[3] = {bb.x + (int)(t % bs.x), bb.y + (int)((t / bs.x) % bs.y),
                         bb.z + (int)(t / ((long long)bs.x * bs.y))};
    double g = 0.0;
    for (int C = 0; C < 3; C++) {
        const int C1 = (C + 1) % 3, C2 = (C + 2) % 3;
        for (int u = 0; u < 2; u++)
            for (int v = 0; v < 2; v++) {
                int e[3] = {cell[0], cell[1], cell[2]};
                e[C1] += u;
                e[C2] += v;
                const long long ri = region_index(p.n, p.per, b0, r, e);
                if (ri < 0) continue;
                int f[3];
                for (int a = 0; a < 3; a++) f[a] = fold(e[a], p.n[a], p.per[a]);
                bool valid = true;
                for (int a = 0; a < 3; a++)
                    if (!p.per[a] && a != C && f[a] == 0) valid = false;
                if (!valid) continue;
                double se = 0.0, ss = 0.0;
                bool pec = false;
                for (int uu = 0; uu < 2; uu++)
                    for (int vv = 0; vv < 2; vv++) {
                        int cc[3] = {f[0], f[1], f[2]};
                        cc[C1] -= 1 - uu;
                        cc[C2] -= 1 - vv;
                        for (int a = 0; a < 3; a++) cc[a] = fold(cc[a], p.n[a], p.per[a]);
                        const MatDev &M = p.mat[p.id[p.slot(cc[0], cc[1], cc[2])]];
                        pec = pec || M.is_pec;
                        se += M.eps_r;
                        ss += M.sigma;
                    }
                if (pec) continue;
                const double eps = p.eps0 * (se / 4), sig = ss / 4;
                const double den = sig / 2.0 + eps / p.dt;
                const double dca = (sig / p.dt) / (den * den), dcb = -(1.0 / p.dt) / (den * den);
                g += (gca[C * tb + ri] * dca + gcb[C * tb + ri] * dcb) * (p.eps0 / 4.0);
            }
    }
    out[t] = g;
}

// ---------------------------------------------------------------------------
// fused schedule: one stencil pass per transposed map
// ---------------------------------------------------------------------------

// E-step coefficients of the edge of family C at slot idx (in the domain):
// ok = false for an edge on a lower wall or with a PEC cell (E' = 0).  The
// mixed-slot case is out of line with scalar arguments (a reference to the
// kernel's parameter block would make the compiler copy it to scratch).
template <typename T>
struct EdgeCoef {
    T ca, cb;
    bool ok;
};

template <typename T>
__device__ __noinline__ EdgeCoef<T> edge_coef_mixed(const uint8_t *id, const MatDev *mat, int n0, int n1, int n2,
                                                     int per0, int per1, int per2, int px, double eps0, double dt,
                                                     int C, int i, int j, int k) {
    const int n[3] = {n0, n1, n2}, per[3] = {per0, per1, per2};
    const int C1 = (C + 1) % 3, C2 = (C + 2) % 3;
    double se = 0.0, ss = 0.0;
    EdgeCoef<T> r{T(0), T(0), false};
    for (int u = 0; u < 2; u++)
        for (int v = 0; v < 2; v++) {
            int cc[3] = {i, j, k};
            cc[C1] -= 1 - u;
            cc[C2] -= 1 - v;
            for (int a = 0; a < 3; a++) cc[a] = fold(cc[a], n[a], per[a]);
            const MatDev &M = mat[id[(long long)cc[0] + (long long)px * ((long long)cc[1] + (long long)n1 * cc[2])]];
            if (M.is_pec) return r;
            se += M.eps_r;
            ss += M.sigma;
        }
    const double eps = eps0 * (se / 4), sig = ss / 4;
    const double den = sig / 2.0 + eps / dt;
    r.ca = (T)(-(sig / 2.0 - eps / dt) / den);
    r.cb = (T)(1.0 / den);
    r.ok = true;
    return r;
}

// the E-step coefficients of the three edges of slot idx (q its slot): one
// class read, then the three table entries together
template <typename T>
__device__ __forceinline__ void edge_coefs(const KParams<T> &p, const int *idx, long long q, T *ca, T *cb, bool *ok) {
    const int cl = p.cls[q];
    ca[0] = ca[1] = ca[2] = cb[0] = cb[1] = cb[2] = T(0);
    ok[0] = ok[1] = ok[2] = false;
    if (cl != kMixed) {
        // the class's packed row (one or two wide loads; a PEC edge has
        // ca = cb = 0, every other edge cb > 0)
        const CoefRow<T> r = coef_row<T>(p.coefv, cl);
#pragma unroll
        for (int C = 0; C < 3; C++) {
            ca[C] = r.ca[C];
            cb[C] = r.cb[C];
            ok[C] = r.cb[C] != T(0);
        }
    }
    // an edge on a lower wall (a non-periodic axis other than its own) is held
    // at zero; a mixed slot's edges read the four cells around them, which
    // exist off the walls only
    for (int C = 0; C < 3; C++) {
        bool wall = false;
        for (int a = 0; a < 3; a++)
            if (a != C && !p.per[a] && idx[a] == 0) wall = true;
        if (wall) {
            ca[C] = cb[C] = T(0);
            ok[C] = false;
        } else if (cl == kMixed) {
            const EdgeCoef<T> r = edge_coef_mixed<T>(p.id, p.mat, p.n[0], p.n[1], p.n[2], p.per[0], p.per[1],
                                                     p.per[2], p.px, p.eps0, p.dt, C, idx[0], idx[1], idx[2]);
            ca[C] = r.ca;
            cb[C] = r.cb;
            ok[C] = r.ok;
        }
    }
}

// the first film whose reach holds the face slot idx, its region index lr
template <typename T>
__device__ __forceinline__ int first_region(const AdjParams<T> &A, const int *idx, long long &lr) {
    for (int f = 0; f < A.p.nfilm; f++) {
        const AdjFilmDev G = scalar_desc(A.af, f);
        const int r0 = idx[0] - G.r0[0], r1 = idx[1] - G.r0[1], r2 = idx[2] - G.r0[2];
        if (r0 >= 0 && r0 < G.rn[0] && r1 >= 0 && r1 < G.rn[1] && r2 >= 0 && r2 < G.rn[2]) {
            lr = (long long)r0 + (long long)G.rn[0] * ((long long)r1 + (long long)G.rn[1] * r2);
            return f;
        }
    }
    return -1;
}

// a neighbour slot t - e_a (D = -1) or t + e_a (D = +1): folded, false when
// outside the domain
template <int D>
__device__ __forceinline__ bool nb(const int *n, const int *per, const int *t, int a, int *q) {
    q[0] = t[0];
    q[1] = t[1];
    q[2] = t[2];
    q[a] = fold(t[a] + D, n[a], per[a]);
    return q[a] >= 0;
}

// the neighbour t + D e_a as nb, or t itself where nb finds none (false):
// the caller evaluates there and drops the value
template <int D>
__device__ __forceinline__ bool nb_or_self(const int *n, const int *per, const int *t, int a, int *q) {
    const bool ok = nb<D>(n, per, t, a, q);
    if (!ok) q[a] = t[a];
    return ok;
}

// the film region's faces: the general face adjoint (magnetic faces, faces
// the solves read), lambda H and lambda M updated in place, the curl-part
// adjoints stored for the field pass
template <typename T>
__global__ void __launch_bounds__(256) k_adj_film_faces(AdjParams<T> A, int f) {
    const AdjFilmDev G = scalar_desc(A.af, f);
    const long long lr = (long long)blockIdx.x * 256 + threadIdx.x;
    if (lr >= G.nr) return;
    const int idx[3] = {G.r0[0] + (int)(lr % G.rn[0]), G.r0[1] + (int)((lr / G.rn[0]) % G.rn[1]),
                        G.r0[2] + (int)(lr / ((long long)G.rn[0] * G.rn[1]))};
    long long l2;
    if (first_region(A, idx, l2) != f) return;
    // one face family per grid row
    T a0, a1;
    const int F = blockIdx.y;
    if (F == 0)
        adj_face_core<T, 0>(A, idx, A.lpsiH[0][1], A.lpsiH[0][2], A.lpsiHo[0][1], A.lpsiHo[0][2], a0, a1);
    else if (F == 1)
        adj_face_core<T, 1>(A, idx, A.lpsiH[1][2], A.lpsiH[1][0], A.lpsiHo[1][2], A.lpsiHo[1][0], a0, a1);
    else
        adj_face_core<T, 2>(A, idx, A.lpsiH[2][0], A.lpsiH[2][1], A.lpsiHo[2][0], A.lpsiHo[2][1], a0, a1);
    G.aDr[(2 * F) * G.nr + lr] = (double)a0;
    G.aDr[(2 * F + 1) * G.nr + lr] = (double)a1;
}

// region index of the folded slot t in the region [b0, b0 + r) (which may
// wrap on a periodic axis), -1 outside
__device__ __forceinline__ long long region_index_folded(const int *n, const int *per, const int *b0, const int *r,
                                                         const int *t) {
    long long li = 0, mul = 1;
    for (int a = 0; a < 3; a++) {
        int loc = t[a] - b0[a];
        if (loc < 0 && per[a]) loc += n[a];
        if (loc < 0 || loc >= r[a]) return -1;
        li += mul * loc;
        mul *= r[a];
    }
    return li;
}

// a new lambda psi value held for a store after the thread's last load
// (q1 / q2 < 0: none)
template <typename T>
struct PsiOut {
    long long q1 = -1, q2 = -1;
    T v1 = T(0), v2 = T(0);
};

// curl-part adjoints (aD0, aD1) of the face of family F at slot f (in the
// domain), general case: from the film region's table, or from lambda H with
// the CPML recursions (own: also store lambda psiH after the map).  In
// float32 every load is unconditional (a lane outside a slab reads its
// lambda H again in place of the slab state and drops it), so that the loads
// of all of a thread's faces can be in flight at once.
template <typename T, int F, int FILM>
__device__ __forceinline__ void hface(const AdjParams<T> &A, const int *f, bool own, T &aD0, T &aD1) {
    constexpr int F1 = (F + 1) % 3, F2 = (F + 2) % 3;
    const KParams<T> &p = A.p;
    if (FILM) {
        long long lr;
        const int fr = first_region(A, f, lr);
        if (fr >= 0) {
            const AdjFilmDev &G = A.af[fr];
            aD0 = (T)G.aDr[(F * 2) * G.nr + lr];
            aD1 = (T)G.aDr[(F * 2 + 1) * G.nr + lr];
            return;
        }
    }
    const T *hp = A.lH[F] + p.slot(f[0], f[1], f[2]);
    const int a1 = f[F1], a2 = f[F2];
    const bool s1 = p.psiH[F][F1] && (a1 < p.nlo[F1] || a1 >= p.n[F1] - p.nhi[F1]);
    const bool s2 = p.psiH[F][F2] && (a2 < p.nlo[F2] || a2 >= p.n[F2] - p.nhi[F2]);
    if constexpr (sizeof(T) == 8) {
        // float64: the slab state loaded where needed only (the unconditional
        // form's registers cost a wave per SIMD here, and it measured slower)
        const T lH = *hp;
        const T g1 = -p.hc * lH, g2 = p.hc * lH;
        aD0 = g1;
        aD1 = g2;
        if (s1) {
            const long long q1 = p.psi_index(F1, f);
            const T aps = A.lpsiH[F][F1][q1] + g1;
            if (own) A.lpsiHo[F][F1][q1] = p.bH[F1][a1] * aps;
            aD0 = g1 + p.cH[F1][a1] * aps;
        }
        if (s2) {
            const long long q2 = p.psi_index(F2, f);
            const T aps = A.lpsiH[F][F2][q2] + g2;
            if (own) A.lpsiHo[F][F2][q2] = p.bH[F2][a2] * aps;
            aD1 = g2 + p.cH[F2][a2] * aps;
        }
    } else {
        const long long q1 = s1 ? p.psi_index(F1, f) : 0, q2 = s2 ? p.psi_index(F2, f) : 0;
        const T lH = *hp;
        const T ps1 = *(s1 ? A.lpsiH[F][F1] + q1 : hp), ps2 = *(s2 ? A.lpsiH[F][F2] + q2 : hp);
        const T b1 = *(s1 ? p.bH[F1] + a1 : hp), c1 = *(s1 ? p.cH[F1] + a1 : hp);
        const T b2 = *(s2 ? p.bH[F2] + a2 : hp), c2 = *(s2 ? p.cH[F2] + a2 : hp);
        const T g1 = -p.hc * lH, g2 = p.hc * lH;
        aD0 = g1;
        aD1 = g2;
        if (s1) {
            const T aps = ps1 + g1;
            if (own) A.lpsiHo[F][F1][q1] = b1 * aps;
            aD0 = g1 + c1 * aps;
        }
        if (s2) {
            const T aps = ps2 + g2;
            if (own) A.lpsiHo[F][F2][q2] = b2 * aps;
            aD1 = g2 + c2 * aps;
        }
    }
}

// float64: a neighbour face of family F at t - e_axis, false past a wall
// (values zero)
template <typename T, int F, int FILM>
__device__ __forceinline__ bool hface_nb(const AdjParams<T> &A, const int *t, int axis, T &x0, T &x1) {
    int u[3];
    if (!nb<-1>(A.p.n, A.p.per, t, axis, u)) {
        x0 = x1 = T(0);
        return false;
    }
    hface<T, F, FILM>(A, u, false, x0, x1);
    return true;
}

// the loss term of the state at the start of the step (film-energy
// gradient, scaled) for the slot t: added to its three lambda E values (in
// registers) and to lambda H of its three faces (film faces: no other thread
// of the pass reads them)
// (PART: 0 both terms, 1 the lambda E term only, 2 the lambda H term only)
template <typename T, int PART = 0>
__device__ __forceinline__ void loss_term(const AdjParams<T> &A, const int *t, long long q, T &l0, T &l1, T &l2) {
    const KParams<T> &p = A.p;
    const FilmDev &F = p.films[A.lfilm];
    const int b0[3] = {F.cb[0], F.cb[1], F.cb[2]}, r[3] = {F.cb[3] + 1, F.cb[4] + 1, F.cb[5] + 1};
    const long long ri = region_index_folded(p.n, p.per, b0, r, t);
    if (ri < 0) return;
    const long long tb = (long long)r[0] * r[1] * r[2];
    T le[3] = {l0, l1, l2};
    for (int C = 0; C < 3; C++) {
        const int C1 = (C + 1) % 3, C2 = (C + 2) % 3;
        double se = 0.0, eps;
        for (int u = 0; u < 2; u++)
            for (int v = 0; v < 2; v++) {
                int cc[3] = {t[0], t[1], t[2]};
                cc[C1] -= u;
                cc[C2] -= v;
                for (int a = 0; a < 3; a++) cc[a] = fold(cc[a], p.n[a], p.per[a]);
                if (cc[0] >= 0 && cc[1] >= 0 && cc[2] >= 0 && film_cell(p, F, cc[0], cc[1], cc[2], eps)) se += eps;
            }
        if (PART != 2 && se != 0.0) le[C] += (T)(A.lscale * p.dV * p.eps0 * se * 0.25 * A.ltape[C * tb + ri]);
        int nc = 0;
        for (int u = 0; u < 2; u++) {
            int cc[3] = {t[0], t[1], t[2]};
            cc[C] -= u;
            for (int a = 0; a < 3; a++) cc[a] = fold(cc[a], p.n[a], p.per[a]);
            if (cc[0] >= 0 && cc[1] >= 0 && cc[2] >= 0 && film_cell(p, F, cc[0], cc[1], cc[2], eps)) nc++;
        }
        if (PART != 1 && nc) A.lH[C][q] += (T)(A.lscale * p.dV * p.mu0 * 0.5 * nc * A.ltape[(3 + C) * tb + ri]);
    }
    l0 = le[0];
    l1 = le[1];
    l2 = le[2];
}

// the flag byte of this block's tile, read through the scalar cache (the
// aligned word that holds it; the table is whole words), so that the wait for
// it does not hold vector loads issued before its first use
__device__ __forceinline__ int adj_tile_flag(const uint8_t *tab) {
    typedef __attribute__((address_space(4))) const uint32_t cword;
    const unsigned ti = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    const uint32_t w = ((cword *)tab)[ti >> 2];
    return (int)((w >> (8 * (ti & 3))) & 0xffu);
}

// the six differences of the transposed curl a slot's half-step pass adds to
// its lambda E, in a tile near a CPML slab (FILM = 0) or a film's reach
// (FILM = 1): d = {d0a, d0b, d1a, d1b, d2a, d2b}, lambda E_C gaining
// dCa + dCb.  Each own face's two curl-part adjoints are paired with their
// neighbours' as soon as those are known, so few values are live at once.
template <typename T, int FILM>
__device__ __forceinline__ void hfield_general(const AdjParams<T> &A, const int *t, T *d) {
    const KParams<T> &p = A.p;
    T a, b, x0, x1;
    bool ok;
    if constexpr (sizeof(T) == 8) {
        // own face of family 1: with the family-1 faces at k - 1 and i - 1
        hface<T, 1, FILM>(A, t, true, a, b);
        ok = hface_nb<T, 1, FILM>(A, t, 2, x0, x1);
        d[0] = dif((ok ? x0 : T(0)) - a, T(0), p.dT[2], p.invd[2]);
        ok = hface_nb<T, 1, FILM>(A, t, 0, x0, x1);
        d[5] = dif((ok ? x1 : T(0)) - b, T(0), p.dT[0], p.invd[0]);
        // family 2: with the family-2 faces at j - 1 and i - 1
        hface<T, 2, FILM>(A, t, true, a, b);
        ok = hface_nb<T, 2, FILM>(A, t, 1, x0, x1);
        d[1] = dif((ok ? x1 : T(0)) - b, T(0), p.dT[1], p.invd[1]);
        ok = hface_nb<T, 2, FILM>(A, t, 0, x0, x1);
        d[2] = dif((ok ? x0 : T(0)) - a, T(0), p.dT[0], p.invd[0]);
        // family 0: with the family-0 faces at k - 1 and j - 1
        hface<T, 0, FILM>(A, t, true, a, b);
        ok = hface_nb<T, 0, FILM>(A, t, 2, x0, x1);
        d[3] = dif((ok ? x1 : T(0)) - b, T(0), p.dT[2], p.invd[2]);
        ok = hface_nb<T, 0, FILM>(A, t, 1, x0, x1);
        d[4] = dif((ok ? x0 : T(0)) - a, T(0), p.dT[1], p.invd[1]);
    } else {
        // the same in float32 with every neighbour evaluated (one past a wall
        // at the own slot, its values dropped): no load waits on a branch
        int u[3];
        hface<T, 1, FILM>(A, t, true, a, b);
        ok = nb_or_self<-1>(p.n, p.per, t, 2, u);
        hface<T, 1, FILM>(A, u, false, x0, x1);
        d[0] = dif((ok ? x0 : T(0)) - a, T(0), p.dT[2], p.invd[2]);
        ok = nb_or_self<-1>(p.n, p.per, t, 0, u);
        hface<T, 1, FILM>(A, u, false, x0, x1);
        d[5] = dif((ok ? x1 : T(0)) - b, T(0), p.dT[0], p.invd[0]);
        hface<T, 2, FILM>(A, t, true, a, b);
        ok = nb_or_self<-1>(p.n, p.per, t, 1, u);
        hface<T, 2, FILM>(A, u, false, x0, x1);
        d[1] = dif((ok ? x1 : T(0)) - b, T(0), p.dT[1], p.invd[1]);
        ok = nb_or_self<-1>(p.n, p.per, t, 0, u);
        hface<T, 2, FILM>(A, u, false, x0, x1);
        d[2] = dif((ok ? x0 : T(0)) - a, T(0), p.dT[0], p.invd[0]);
        hface<T, 0, FILM>(A, t, true, a, b);
        ok = nb_or_self<-1>(p.n, p.per, t, 2, u);
        hface<T, 0, FILM>(A, u, false, x0, x1);
        d[3] = dif((ok ? x1 : T(0)) - b, T(0), p.dT[2], p.invd[2]);
        ok = nb_or_self<-1>(p.n, p.per, t, 1, u);
        hface<T, 0, FILM>(A, u, false, x0, x1);
        d[4] = dif((ok ? x0 : T(0)) - a, T(0), p.dT[1], p.invd[1]);
    }
}

// ---------------------------------------------------------------------------
// The merged pass of two consecutive half-step transposes on the E side: the
// first half step of step m (with the E step's lambda E = ca lambda E', the
// eps-box sums, the loss term's lambda E part and a weighted trace's term of
// the state at step m's start), then the second half step of step m - 1,
// whose lambda H of non-film faces is the same (the first pass changes lambda
// E only; the film kernels between them change the film region's faces,
// which both take from their own tables).  A face's CPML state goes through
// both recursions in one thread (read from set lpsiH, stored in lpsiHo);
// every value follows the two single passes' operation sequence, so the
// results are theirs, bitwise.  Used only where no film's reach meets a CPML
// slab (the film-region passes keep their state per half step).
// ---------------------------------------------------------------------------

// the two half steps' curl-part adjoints (a0, a1: the first; b0, b1: the
// second) of the face of family F at slot f; own: store its lambda psiH after
// both maps
template <typename T, int F, int FILM>
__device__ __forceinline__ void hface2(const AdjParams<T> &A, const int *f, bool own, T &a0, T &a1, T &b0, T &b1) {
    constexpr int F1 = (F + 1) % 3, F2 = (F + 2) % 3;
    const KParams<T> &p = A.p;
    if (FILM) {
        long long lr;
        const int fr = first_region(A, f, lr);
        if (fr >= 0) {
            const AdjFilmDev G = scalar_desc(A.af, fr), Gb = scalar_desc(A.afb, fr);
            a0 = (T)G.aDr[(F * 2) * G.nr + lr];
            a1 = (T)G.aDr[(F * 2 + 1) * G.nr + lr];
            b0 = (T)Gb.aDr[(F * 2) * Gb.nr + lr];
            b1 = (T)Gb.aDr[(F * 2 + 1) * Gb.nr + lr];
            return;
        }
    }
    const T lH = A.lH[F][p.slot(f[0], f[1], f[2])];
    const T g1 = -p.hc * lH, g2 = p.hc * lH;
    a0 = b0 = g1;
    a1 = b1 = g2;
    const int c1 = f[F1], c2 = f[F2];
    if (p.psiH[F][F1] && (c1 < p.nlo[F1] || c1 >= p.n[F1] - p.nhi[F1])) {
        const long long qq = p.psi_index(F1, f);
        const T bb = p.bH[F1][c1], cc = p.cH[F1][c1];
        const T aps = A.lpsiH[F][F1][qq] + g1;
        a0 = g1 + cc * aps;
        const T aps2 = bb * aps + g1;
        b0 = g1 + cc * aps2;
        if (own) A.lpsiHo[F][F1][qq] = bb * aps2;
    }
    if (p.psiH[F][F2] && (c2 < p.nlo[F2] || c2 >= p.n[F2] - p.nhi[F2])) {
        const long long qq = p.psi_index(F2, f);
        const T bb = p.bH[F2][c2], cc = p.cH[F2][c2];
        const T aps = A.lpsiH[F][F2][qq] + g2;
        a1 = g2 + cc * aps;
        const T aps2 = bb * aps + g2;
        b1 = g2 + cc * aps2;
        if (own) A.lpsiHo[F][F2][qq] = bb * aps2;
    }
}

// the six differences of each half step (d: the first, e: the second), as
// hfield_general's
template <typename T, int FILM>
__device__ __forceinline__ void hfield_general2(const AdjParams<T> &A, const int *t, T *d, T *e) {
    const KParams<T> &p = A.p;
    T a0, a1, b0, b1, x0, x1, y0, y1;
    int u[3];
    bool ok;
    // own face of family 1: with the family-1 faces at k - 1 and i - 1
    hface2<T, 1, FILM>(A, t, true, a0, a1, b0, b1);
    ok = nb_or_self<-1>(p.n, p.per, t, 2, u);
    hface2<T, 1, FILM>(A, u, false, x0, x1, y0, y1);
    d[0] = dif((ok ? x0 : T(0)) - a0, T(0), p.dT[2], p.invd[2]);
    e[0] = dif((ok ? y0 : T(0)) - b0, T(0), p.dT[2], p.invd[2]);
    ok = nb_or_self<-1>(p.n, p.per, t, 0, u);
    hface2<T, 1, FILM>(A, u, false, x0, x1, y0, y1);
    d[5] = dif((ok ? x1 : T(0)) - a1, T(0), p.dT[0], p.invd[0]);
    e[5] = dif((ok ? y1 : T(0)) - b1, T(0), p.dT[0], p.invd[0]);
    // family 2: with the family-2 faces at j - 1 and i - 1
    hface2<T, 2, FILM>(A, t, true, a0, a1, b0, b1);
    ok = nb_or_self<-1>(p.n, p.per, t, 1, u);
    hface2<T, 2, FILM>(A, u, false, x0, x1, y0, y1);
    d[1] = dif((ok ? x1 : T(0)) - a1, T(0), p.dT[1], p.invd[1]);
    e[1] = dif((ok ? y1 : T(0)) - b1, T(0), p.dT[1], p.invd[1]);
    ok = nb_or_self<-1>(p.n, p.per, t, 0, u);
    hface2<T, 2, FILM>(A, u, false, x0, x1, y0, y1);
    d[2] = dif((ok ? x0 : T(0)) - a0, T(0), p.dT[0], p.invd[0]);
    e[2] = dif((ok ? y0 : T(0)) - b0, T(0), p.dT[0], p.invd[0]);
    // family 0: with the family-0 faces at k - 1 and j - 1
    hface2<T, 0, FILM>(A, t, true, a0, a1, b0, b1);
    ok = nb_or_self<-1>(p.n, p.per, t, 2, u);
    hface2<T, 0, FILM>(A, u, false, x0, x1, y0, y1);
    d[3] = dif((ok ? x1 : T(0)) - a1, T(0), p.dT[2], p.invd[2]);
    e[3] = dif((ok ? y1 : T(0)) - b1, T(0), p.dT[2], p.invd[2]);
    ok = nb_or_self<-1>(p.n, p.per, t, 1, u);
    hface2<T, 0, FILM>(A, u, false, x0, x1, y0, y1);
    d[4] = dif((ok ? x0 : T(0)) - a0, T(0), p.dT[1], p.invd[1]);
    e[4] = dif((ok ? y0 : T(0)) - b0, T(0), p.dT[1], p.invd[1]);
}

template <typename T>
__global__ void __launch_bounds__(256) k_adj_hfield2(AdjParams<T> A) {
    const KParams<T> &p = A.p;
    const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y, k = blockIdx.z;
    if (i >= p.n[0] || j >= p.n[1]) return;
    const int t[3] = {i, j, k};
    const long long q = p.slot(i, j, k);
    const uint8_t fl = (uint8_t)adj_tile_flag(A.aflags);
    // the slot's lambda E is touched once per pass: non-temporal (the lambda
    // H the neighbouring slots read again stays in L2)
    T l0 = __builtin_nontemporal_load(A.lE[0] + q), l1 = __builtin_nontemporal_load(A.lE[1] + q),
      l2 = __builtin_nontemporal_load(A.lE[2] + q);
    T ca[3], cb[3];
    bool ok[3];
    edge_coefs<T>(p, t, q, ca, cb, ok);
    T dd[6], de[6];
    if (fl == 0) {
        // no CPML state, no film region: both half steps take -/+ hc lambda H
        T o0[3], o1[3];
        T n1m2 = T(0), n2m1 = T(0), n2m0 = T(0), n0m2 = T(0), n0m1 = T(0), n1m0 = T(0);
        int u[3];
#pragma unroll
        for (int F = 0; F < 3; F++) {
            const T l = A.lH[F][q];
            o0[F] = -(p.hc * l);
            o1[F] = p.hc * l;
        }
        bool ok2 = nb_or_self<-1>(p.n, p.per, t, 2, u);
        const T h1m2 = A.lH[1][p.slot(u[0], u[1], u[2])], h0m2 = A.lH[0][p.slot(u[0], u[1], u[2])];
        bool ok1 = nb_or_self<-1>(p.n, p.per, t, 1, u);
        const T h2m1 = A.lH[2][p.slot(u[0], u[1], u[2])], h0m1 = A.lH[0][p.slot(u[0], u[1], u[2])];
        bool ok0 = nb_or_self<-1>(p.n, p.per, t, 0, u);
        const T h2m0 = A.lH[2][p.slot(u[0], u[1], u[2])], h1m0 = A.lH[1][p.slot(u[0], u[1], u[2])];
        if (ok2) {
            n1m2 = -(p.hc * h1m2);
            n0m2 = p.hc * h0m2;
        }
        if (ok1) {
            n2m1 = p.hc * h2m1;
            n0m1 = -(p.hc * h0m1);
        }
        if (ok0) {
            n2m0 = -(p.hc * h2m0);
            n1m0 = p.hc * h1m0;
        }
        dd[0] = dif(n1m2 - o0[1], T(0), p.dT[2], p.invd[2]);
        dd[1] = dif(n2m1 - o1[2], T(0), p.dT[1], p.invd[1]);
        dd[2] = dif(n2m0 - o0[2], T(0), p.dT[0], p.invd[0]);
        dd[3] = dif(n0m2 - o1[0], T(0), p.dT[2], p.invd[2]);
        dd[4] = dif(n0m1 - o0[0], T(0), p.dT[1], p.invd[1]);
        dd[5] = dif(n1m0 - o1[1], T(0), p.dT[0], p.invd[0]);
#pragma unroll
        for (int w = 0; w < 6; w++) de[w] = dd[w];
    } else if (fl & 4) {
        hfield_general2<T, 1>(A, t, dd, de);
    } else {
        hfield_general2<T, 0>(A, t, dd, de);
    }
    if (A.btape) {
        // dL/dca += lambda E' E^n, dL/dcb += lambda E' x^n over the eps box
        const int r[3] = {A.bs[0] + 1, A.bs[1] + 1, A.bs[2] + 1};
        const long long ri = region_index_folded(p.n, p.per, A.bb, r, t);
        if (ri >= 0) {
            const long long tb = (long long)r[0] * r[1] * r[2];
            const T lv[3] = {l0, l1, l2};
#pragma unroll
            for (int C = 0; C < 3; C++) {
                A.gca_box[C * tb + ri] += (double)lv[C] * A.btape[C * tb + ri];
                A.gcb_box[C * tb + ri] += (double)lv[C] * A.btape[(3 + C) * tb + ri];
            }
        }
    }
    // the first half step of step m (the E step's scaling first)
    l0 = ok[0] ? ca[0] * l0 : T(0);
    l1 = ok[1] ? ca[1] * l1 : T(0);
    l2 = ok[2] ? ca[2] * l2 : T(0);
    l0 = l0 + (dd[0] + dd[1]);
    l1 = l1 + (dd[2] + dd[3]);
    l2 = l2 + (dd[4] + dd[5]);
    if (A.ltape && (fl & 4) && A.seg0[0] + A.m > A.loss_from) loss_term<T, 1>(A, t, q, l0, l1, l2);
    if (A.pw && q == A.pw_slot) {
        const long long n = A.seg0[0] + A.m;
        if (n >= 1) {
            const T v = (T)(A.pw_scale * A.pw[n - 1]);
            if (A.pw_comp == 0)
                l0 += v;
            else if (A.pw_comp == 1)
                l1 += v;
            else
                l2 += v;
        }
    }
    // the second half step of step m - 1
    l0 = l0 + (de[0] + de[1]);
    l1 = l1 + (de[2] + de[3]);
    l2 = l2 + (de[4] + de[5]);
    __builtin_nontemporal_store(l0, A.lE[0] + q);
    __builtin_nontemporal_store(l1, A.lE[1] + q);
    __builtin_nontemporal_store(l2, A.lE[2] + q);
    A.mu[0][q] = ok[0] ? cb[0] * l0 : T(0);
    A.mu[1][q] = ok[1] ? cb[1] * l1 : T(0);
    A.mu[2][q] = ok[2] ? cb[2] * l2 : T(0);
}

// the loss term's lambda H part of the state at step m's start, for the film
// region's faces (before the film kernels of the next half step read them)
template <typename T>
__global__ void __launch_bounds__(256) k_adj_loss_h(AdjParams<T> A) {
    const KParams<T> &p = A.p;
    if (!(A.seg0[0] + A.m > A.loss_from)) return;
    const FilmDev F = film_desc(p.films, A.lfilm);
    const int r[3] = {F.cb[3] + 1, F.cb[4] + 1, F.cb[5] + 1};
    const long long lr = (long long)blockIdx.x * 256 + threadIdx.x;
    if (lr >= (long long)r[0] * r[1] * r[2]) return;
    int t[3] = {F.cb[0] + (int)(lr % r[0]), F.cb[1] + (int)((lr / r[0]) % r[1]),
                F.cb[2] + (int)(lr / ((long long)r[0] * r[1]))};
    for (int a = 0; a < 3; a++) {
        if (t[a] >= p.n[a] && p.per[a]) t[a] -= p.n[a];
        if (t[a] >= p.n[a]) return;
    }
    T l0 = T(0), l1 = T(0), l2 = T(0);
    loss_term<T, 2>(A, t, p.slot(t[0], t[1], t[2]), l0, l1, l2);
}

// the transposed half step on the E side: lambda E_C += the transposed curl
// of the faces' curl-part adjoints (lambda E = ca lambda E' first when SCALE)
template <typename T, int SCALE>
__global__ void __launch_bounds__(256) k_adj_hfield(AdjParams<T> A) {
    const KParams<T> &p = A.p;
    const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y, k = blockIdx.z;
    if (i >= p.n[0] || j >= p.n[1]) return;
    const int t[3] = {i, j, k};
    const long long q = p.slot(i, j, k);
    const uint8_t fl = (uint8_t)adj_tile_flag(A.aflags);
    // lambda E and the edge coefficients (one class read) before the faces
    T l0 = A.lE[0][q], l1 = A.lE[1][q], l2 = A.lE[2][q];
    T ca[3], cb[3];
    bool ok[3];
    edge_coefs<T>(p, t, q, ca, cb, ok);
    const T ca0 = ca[0], cb0 = cb[0], ca1 = ca[1], cb1 = cb[1], ca2 = ca[2], cb2 = cb[2];
    const bool v0 = ok[0], v1 = ok[1], v2 = ok[2];
    // dd: the transposed curl's six differences (see hfield_general)
    T dd[6];
    if (fl == 0) {
        // own faces: aD0, aD1 of each family; neighbours, named by family
        // and the axis of the -1 offset
        T o0[3], o1[3];
        T n1m2 = T(0), n2m1 = T(0), n2m0 = T(0), n0m2 = T(0), n0m1 = T(0), n1m0 = T(0);
        int u[3];
#pragma unroll
        for (int F = 0; F < 3; F++) {
            const T l = A.lH[F][q];
            o0[F] = -(p.hc * l);
            o1[F] = p.hc * l;
        }
        if constexpr (sizeof(T) == 8) {
            if (nb<-1>(p.n, p.per, t, 2, u)) n1m2 = -(p.hc * A.lH[1][p.slot(u[0], u[1], u[2])]);
            if (nb<-1>(p.n, p.per, t, 1, u)) n2m1 = p.hc * A.lH[2][p.slot(u[0], u[1], u[2])];
            if (nb<-1>(p.n, p.per, t, 0, u)) n2m0 = -(p.hc * A.lH[2][p.slot(u[0], u[1], u[2])]);
            if (nb<-1>(p.n, p.per, t, 2, u)) n0m2 = p.hc * A.lH[0][p.slot(u[0], u[1], u[2])];
            if (nb<-1>(p.n, p.per, t, 1, u)) n0m1 = -(p.hc * A.lH[0][p.slot(u[0], u[1], u[2])]);
            if (nb<-1>(p.n, p.per, t, 0, u)) n1m0 = p.hc * A.lH[1][p.slot(u[0], u[1], u[2])];
        } else {
            // the neighbours' lambda H (a wall's read at the own slot and dropped)
            bool ok2 = nb_or_self<-1>(p.n, p.per, t, 2, u);
            const T h1m2 = A.lH[1][p.slot(u[0], u[1], u[2])], h0m2 = A.lH[0][p.slot(u[0], u[1], u[2])];
            bool ok1 = nb_or_self<-1>(p.n, p.per, t, 1, u);
            const T h2m1 = A.lH[2][p.slot(u[0], u[1], u[2])], h0m1 = A.lH[0][p.slot(u[0], u[1], u[2])];
            bool ok0 = nb_or_self<-1>(p.n, p.per, t, 0, u);
            const T h2m0 = A.lH[2][p.slot(u[0], u[1], u[2])], h1m0 = A.lH[1][p.slot(u[0], u[1], u[2])];
            if (ok2) {
                n1m2 = -(p.hc * h1m2);
                n0m2 = p.hc * h0m2;
            }
            if (ok1) {
                n2m1 = p.hc * h2m1;
                n0m1 = -(p.hc * h0m1);
            }
            if (ok0) {
                n2m0 = -(p.hc * h2m0);
                n1m0 = p.hc * h1m0;
            }
        }
        dd[0] = dif(n1m2 - o0[1], T(0), p.dT[2], p.invd[2]);
        dd[1] = dif(n2m1 - o1[2], T(0), p.dT[1], p.invd[1]);
        dd[2] = dif(n2m0 - o0[2], T(0), p.dT[0], p.invd[0]);
        dd[3] = dif(n0m2 - o1[0], T(0), p.dT[2], p.invd[2]);
        dd[4] = dif(n0m1 - o0[0], T(0), p.dT[1], p.invd[1]);
        dd[5] = dif(n1m0 - o1[1], T(0), p.dT[0], p.invd[0]);
    } else if (fl & 4) {
        hfield_general<T, 1>(A, t, dd);
    } else {
        hfield_general<T, 0>(A, t, dd);
    }
    if (SCALE && A.btape) {
        // dL/dca += lambda E' E^n, dL/dcb += lambda E' x^n over the eps box
        const int r[3] = {A.bs[0] + 1, A.bs[1] + 1, A.bs[2] + 1};
        const long long ri = region_index_folded(p.n, p.per, A.bb, r, t);
        if (ri >= 0) {
            const long long tb = (long long)r[0] * r[1] * r[2];
            const T lv[3] = {l0, l1, l2};
#pragma unroll
            for (int C = 0; C < 3; C++) {
                A.gca_box[C * tb + ri] += (double)lv[C] * A.btape[C * tb + ri];
                A.gcb_box[C * tb + ri] += (double)lv[C] * A.btape[(3 + C) * tb + ri];
            }
        }
    }
    if (SCALE) {
        l0 = v0 ? ca0 * l0 : T(0);
        l1 = v1 ? ca1 * l1 : T(0);
        l2 = v2 ? ca2 * l2 : T(0);
    }
    l0 = l0 + (dd[0] + dd[1]);
    l1 = l1 + (dd[2] + dd[3]);
    l2 = l2 + (dd[4] + dd[5]);
    if (SCALE && A.ltape && (fl & 4) && A.seg0[0] + A.m > A.loss_from)
        loss_term(A, t, q, l0, l1, l2);
    if (SCALE && A.pw && q == A.pw_slot) {
        // the weighted trace's term of the state at the step's start (time n)
        const long long n = A.seg0[0] + A.m;
        if (n >= 1) {
            const T v = (T)(A.pw_scale * A.pw[n - 1]);
            if (A.pw_comp == 0)
                l0 += v;
            else if (A.pw_comp == 1)
                l1 += v;
            else
                l2 += v;
        }
    }
    A.lE[0][q] = l0;
    A.lE[1][q] = l1;
    A.lE[2][q] = l2;
    if (!SCALE) {
        // the E-step adjoint's input: cb lambda E' (zero on a wall or PEC edge)
        A.mu[0][q] = v0 ? cb0 * l0 : T(0);
        A.mu[1][q] = v1 ? cb1 * l1 : T(0);
        A.mu[2][q] = v2 ? cb2 * l2 : T(0);
    }
}

// curl-part adjoints (eD0, eD1) of the E edge of family X at slot e (in the
// domain): mu = cb lambda E' with the CPML recursions along X+1 (in1 -> out1)
// and X+2 (in2 -> out2); own: store lambda psiE after the map.  (On a wall or
// PEC edge mu is zero, and so stays its lambda psiE.)
template <typename T, int X, int PML>
__device__ __forceinline__ void eedge(const AdjParams<T> &A, const int *e, const T *in1, const T *in2, PsiOut<T> *own,
                                      T &eD0, T &eD1) {
    constexpr int X1 = (X + 1) % 3, X2 = (X + 2) % 3;
    const KParams<T> &p = A.p;
    const T *mp = A.mu[X] + p.slot(e[0], e[1], e[2]);
    const T lx = *mp;
    eD0 = lx;
    eD1 = -lx;
    if (PML) {
        const int a1 = e[X1], a2 = e[X2];
        const bool s1 = p.psiE[X][X1] && (a1 < p.nlo[X1] || a1 >= p.n[X1] - p.nhi[X1]);
        const bool s2 = p.psiE[X][X2] && (a2 < p.nlo[X2] || a2 >= p.n[X2] - p.nhi[X2]);
        if constexpr (sizeof(T) == 8) {
            // float64: the slab state loaded where needed only (fewer registers)
            if (s1) {
                const long long q1 = p.psi_index(X1, e);
                const T aps = in1[q1] + lx;
                if (own) {
                    own->q1 = q1;
                    own->v1 = p.bE[X1][a1] * aps;
                }
                eD0 = lx + p.cE[X1][a1] * aps;
            }
            if (s2) {
                const long long q2 = p.psi_index(X2, e);
                const T aps = in2[q2] - lx;
                if (own) {
                    own->q2 = q2;
                    own->v2 = p.bE[X2][a2] * aps;
                }
                eD1 = -lx + p.cE[X2][a2] * aps;
            }
        } else {
            // float32: unconditional loads (a lane outside a slab reads mu again
            // and drops it), so that the loads of all of a thread's edges are in
            // flight at once
            const long long q1 = s1 ? p.psi_index(X1, e) : 0, q2 = s2 ? p.psi_index(X2, e) : 0;
            const T ps1 = *(s1 ? in1 + q1 : mp), ps2 = *(s2 ? in2 + q2 : mp);
            const T b1 = *(s1 ? p.bE[X1] + a1 : mp), c1 = *(s1 ? p.cE[X1] + a1 : mp);
            const T b2 = *(s2 ? p.bE[X2] + a2 : mp), c2 = *(s2 ? p.cE[X2] + a2 : mp);
            if (s1) {
                const T aps = ps1 + lx;
                if (own) {
                    own->q1 = q1;
                    own->v1 = b1 * aps;
                }
                eD0 = lx + c1 * aps;
            }
            if (s2) {
                const T aps = ps2 - lx;
                if (own) {
                    own->q2 = q2;
                    own->v2 = b2 * aps;
                }
                eD1 = -lx + c2 * aps;
            }
        }
    }
}

// a neighbour edge of family X at t + e_axis: false past a wall (values
// zero); float32 evaluates at the own slot there and drops the values (no
// load waits on a branch), float64 branches (fewer registers)
template <typename T, int X, int PML>
__device__ __forceinline__ bool eedge_nb(const AdjParams<T> &A, const int *t, int axis, const T *in1, const T *in2,
                                         T &x0, T &x1) {
    int u[3];
    if constexpr (sizeof(T) == 8) {
        if (!nb<1>(A.p.n, A.p.per, t, axis, u)) {
            x0 = x1 = T(0);
            return false;
        }
        eedge<T, X, PML>(A, u, in1, in2, nullptr, x0, x1);
        return true;
    } else {
        const bool ok = nb_or_self<1>(A.p.n, A.p.per, t, axis, u);
        eedge<T, X, PML>(A, u, in1, in2, nullptr, x0, x1);
        return ok;
    }
}

// the transposed E step on the H side: lambda H_C += the transposed curl of
// the edges' curl-part adjoints; lambda E' itself is scaled by ca in the
// next half-step pass
template <typename T, int PML>
__device__ __forceinline__ void efield_body(const AdjParams<T> &A, const int *t, long long q) {
    const KParams<T> &p = A.p;
    const bool par = PML ? (((A.seg0[0] + A.m) & 1) != 0) : false;
    // lambda psiE of step n: read set n & 1, write the other (one select per
    // pointer: indexing the parameter block through a pointer would copy it
    // to scratch)
    const T *i0a = par ? A.lpsiE2[0][1] : A.lpsiE[0][1], *i0b = par ? A.lpsiE2[0][2] : A.lpsiE[0][2];
    const T *i1a = par ? A.lpsiE2[1][2] : A.lpsiE[1][2], *i1b = par ? A.lpsiE2[1][0] : A.lpsiE[1][0];
    const T *i2a = par ? A.lpsiE2[2][0] : A.lpsiE[2][0], *i2b = par ? A.lpsiE2[2][1] : A.lpsiE[2][1];
    // every load of the thread before any store: lambda H of the slot, then
    // the edges (own edges' new lambda psiE held until the end; the sets read
    // and written are different arrays)
    // (the slot's lambda H is touched once per pass: non-temporal; the mu
    // the neighbouring edges read again stays in L2)
    const T lh0 = __builtin_nontemporal_load(A.lH[0] + q), lh1 = __builtin_nontemporal_load(A.lH[1] + q),
            lh2 = __builtin_nontemporal_load(A.lH[2] + q);
    PsiOut<T> w0, w1, w2;
    T o0[3], o1[3], x0, x1;
    eedge<T, 0, PML>(A, t, i0a, i0b, PML ? &w0 : nullptr, o0[0], o1[0]);
    eedge<T, 1, PML>(A, t, i1a, i1b, PML ? &w1 : nullptr, o0[1], o1[1]);
    eedge<T, 2, PML>(A, t, i2a, i2b, PML ? &w2 : nullptr, o0[2], o1[2]);
    T n1p2 = T(0), n2p1 = T(0), n2p0 = T(0), n0p2 = T(0), n0p1 = T(0), n1p0 = T(0);
    // the +1 neighbours' edges
    if (eedge_nb<T, 1, PML>(A, t, 2, i1a, i1b, x0, x1)) n1p2 = x0;
    if (eedge_nb<T, 0, PML>(A, t, 2, i0a, i0b, x0, x1)) n0p2 = x1;
    if (eedge_nb<T, 2, PML>(A, t, 1, i2a, i2b, x0, x1)) n2p1 = x1;
    if (eedge_nb<T, 0, PML>(A, t, 1, i0a, i0b, x0, x1)) n0p1 = x0;
    if (eedge_nb<T, 2, PML>(A, t, 0, i2a, i2b, x0, x1)) n2p0 = x0;
    if (eedge_nb<T, 1, PML>(A, t, 0, i1a, i1b, x0, x1)) n1p0 = x1;
    if (PML) {
        T *o0a = par ? A.lpsiE[0][1] : A.lpsiE2[0][1], *o0b = par ? A.lpsiE[0][2] : A.lpsiE2[0][2];
        T *o1a = par ? A.lpsiE[1][2] : A.lpsiE2[1][2], *o1b = par ? A.lpsiE[1][0] : A.lpsiE2[1][0];
        T *o2a = par ? A.lpsiE[2][0] : A.lpsiE2[2][0], *o2b = par ? A.lpsiE[2][1] : A.lpsiE2[2][1];
        if (w0.q1 >= 0) o0a[w0.q1] = w0.v1;
        if (w0.q2 >= 0) o0b[w0.q2] = w0.v2;
        if (w1.q1 >= 0) o1a[w1.q1] = w1.v1;
        if (w1.q2 >= 0) o1b[w1.q2] = w1.v2;
        if (w2.q1 >= 0) o2a[w2.q1] = w2.v1;
        if (w2.q2 >= 0) o2b[w2.q2] = w2.v2;
    }
    __builtin_nontemporal_store(
        lh0 + (dif(o0[1] - n1p2, T(0), p.dT[2], p.invd[2]) + dif(o1[2] - n2p1, T(0), p.dT[1], p.invd[1])), A.lH[0] + q);
    __builtin_nontemporal_store(
        lh1 + (dif(o0[2] - n2p0, T(0), p.dT[0], p.invd[0]) + dif(o1[0] - n0p2, T(0), p.dT[2], p.invd[2])), A.lH[1] + q);
    __builtin_nontemporal_store(
        lh2 + (dif(o0[0] - n0p1, T(0), p.dT[1], p.invd[1]) + dif(o1[1] - n1p0, T(0), p.dT[0], p.invd[0])), A.lH[2] + q);
}

template <typename T>
__global__ void __launch_bounds__(256) k_adj_efield(AdjParams<T> A) {
    const KParams<T> &p = A.p;
    const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y, k = blockIdx.z;
    if (i >= p.n[0] || j >= p.n[1]) return;
    const int t[3] = {i, j, k};
    const long long q = p.slot(i, j, k);
    if (adj_tile_flag(A.aflags) & 1)
        efield_body<T, 1>(A, t, q);
    else
        efield_body<T, 0>(A, t, q);
}

__global__ void __launch_bounds__(256) k_copy_segs(const CopySeg *segs) {
    const CopySeg S = segs[blockIdx.y];
    const long long n16 = S.bytes >> 4;
    const uint4 *src = (const uint4 *)S.src;
    uint4 *dst = (uint4 *)S.dst;
    const long long stride = (long long)gridDim.x * 256;
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < n16; t += stride) dst[t] = src[t];
    const long long rem = (S.bytes - (n16 << 4)) >> 2;
    if (blockIdx.x == 0 && threadIdx.x < rem)
        ((uint32_t *)S.dst)[n16 * 4 + threadIdx.x] = ((const uint32_t *)S.src)[n16 * 4 + threadIdx.x];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static dim3 slot_grid(const int *n) { return dim3((n[0] + 63) / 64, (n[1] + 3) / 4, n[2]); }

// lambda of the state before a half step from lambda after it; the B^
// prepass of the input state must have run (launch_film phase-1 prepass)
template <typename T>
hipError_t launch_adj_half(const AdjParams<T> &A, int nblk, hipStream_t s) {
    if (nblk) k_adj_film<T><<<dim3(nblk), dim3(256), 0, s>>>(A);
    k_adj_face<T><<<slot_grid(A.p.n), dim3(64, 4), 0, s>>>(A);
    if (nblk) k_adj_film_commit<<<dim3(nblk), dim3(256), 0, s>>>(A.p.blocktab, A.p.films, A.af);
    k_adj_curlE<T><<<slot_grid(A.p.n), dim3(64, 4), 0, s>>>(A);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_estep(const AdjParams<T> &A, hipStream_t s) {
    k_adj_estep<T><<<slot_grid(A.p.n), dim3(64, 4), 0, s>>>(A);
    k_adj_curlH<T><<<slot_grid(A.p.n), dim3(64, 4), 0, s>>>(A);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_loss(const AdjParams<T> &A, int film, double scale, hipStream_t s) {
    k_adj_loss<T><<<slot_grid(A.p.n), dim3(64, 4), 0, s>>>(A, film, scale);
    return hipGetLastError();
}

hipError_t launch_adj_init_ms(const int4 *blocktab, int nblk, const FilmDev *films, const AdjFilmDev *af,
                              const double *u, hipStream_t s) {
    if (nblk) k_adj_init_ms<<<dim3(nblk), dim3(256), 0, s>>>(blocktab, films, af, u[0], u[1], u[2]);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_film_energy(const KParams<T> &p, int film, double *part, double *acc, double scale, hipStream_t s) {
    const dim3 g = slot_grid(p.n);
    k_film_energy<T><<<g, dim3(64, 4), 0, s>>>(p, film, part);
    k_accum<<<dim3(1), dim3(64), 0, s>>>(part, (int)(g.x * g.y * g.z), acc, scale);
    return hipGetLastError();
}

hipError_t launch_set_step(long long *step, long long v, hipStream_t s) {
    k_set_step<<<dim3(1), dim3(64), 0, s>>>(step, v);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_eps(const AdjParams<T> &A, const int *box, double *out, hipStream_t s) {
    const long long nc = (long long)box[3] * box[4] * box[5];
    if (nc == 0) return hipSuccess;
    k_adj_eps<T><<<dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s>>>(
        A, make_int4(box[0], box[1], box[2], 0), make_int4(box[3], box[4], box[5], 0), out);
    return hipGetLastError();
}

long long film_tape_size(const int *cb) { return 6LL * (cb[3] + 1) * (cb[4] + 1) * (cb[5] + 1); }
long long box_tape_size(const int *box) { return 6LL * (box[3] + 1) * (box[4] + 1) * (box[5] + 1); }

// cb: the film's cell box (it sizes the grid)
template <typename T>
hipError_t launch_tape_loss(const KParams<T> &p, int film, int merged, double *dst, hipStream_t s, const int *cb) {
    const long long tb = film_tape_size(cb) / 6;
    k_tape_loss<T><<<dim3((unsigned)((tb + 255) / 256)), dim3(256), 0, s>>>(p, film, merged, dst);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_loss_tape(const AdjParams<T> &A, int film, double scale, const double *tape,
                                const long long *seg0, int m, long long loss_from, hipStream_t s, const int *cb) {
    const long long tb = film_tape_size(cb) / 6;
    k_adj_loss_tape<T><<<dim3((unsigned)((tb + 255) / 256)), dim3(256), 0, s>>>(A, film, scale, tape, seg0, m,
                                                                               loss_from);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_loss_eps_tape(const KParams<T> &p, int film, double scale, const double *tape,
                                    const long long *seg0, int m, long long loss_from, double *acc, hipStream_t s,
                                    const int *cb) {
    const long long nc = (long long)cb[3] * cb[4] * cb[5];
    k_adj_loss_eps_tape<T><<<dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s>>>(p, film, scale, tape, seg0, m,
                                                                                    loss_from, acc);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_loss_eps_state(const KParams<T> &p, int film, double scale, double *acc, hipStream_t s,
                                     const int *cb) {
    const long long nc = (long long)cb[3] * cb[4] * cb[5];
    k_adj_loss_eps_state<T><<<dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s>>>(p, film, scale, acc);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_tape_box(const KParams<T> &p, const int *box, double *dst, hipStream_t s) {
    const long long tb = box_tape_size(box) / 6;
    k_tape_box<T><<<dim3((unsigned)((tb + 255) / 256)), dim3(256), 0, s>>>(
        p, make_int4(box[0], box[1], box[2], 0), make_int4(box[3], box[4], box[5], 0), dst);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_eps_box(const KParams<T> &p, const int *box, const double *gca, const double *gcb, double *out,
                              hipStream_t s) {
    const long long nc = (long long)box[3] * box[4] * box[5];
    if (nc == 0) return hipSuccess;
    k_adj_eps_box<T><<<dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s>>>(
        p, make_int4(box[0], box[1], box[2], 0), make_int4(box[3], box[4], box[5], 0), gca, gcb, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_half_fused(const AdjParams<T> &A, int nblk, int scale, const long long *film_nr,
                                 hipStream_t s) {
    if (nblk) k_adj_film<T><<<dim3(nblk), dim3(256), 0, s>>>(A);
    for (int f = 0; f < A.p.nfilm; f++)
        if (film_nr[f] > 0)
            k_adj_film_faces<T><<<dim3((unsigned)((film_nr[f] + 255) / 256), 3), dim3(256), 0, s>>>(A, f);
    if (scale)
        k_adj_hfield<T, 1><<<slot_grid(A.p.n), dim3(64, 4), 0, s>>>(A);
    else
        k_adj_hfield<T, 0><<<slot_grid(A.p.n), dim3(64, 4), 0, s>>>(A);
    return hipGetLastError();
}

// the film part of a half-step transpose (the magnetic faces' LLG transpose,
// the film reach's faces and their table), then the merged field pass
template <typename T>
hipError_t launch_adj_film_part(const AdjParams<T> &A, int nblk, const long long *film_nr, hipStream_t s) {
    if (nblk) k_adj_film<T><<<dim3(nblk), dim3(256), 0, s>>>(A);
    for (int f = 0; f < A.p.nfilm; f++)
        if (film_nr[f] > 0)
            k_adj_film_faces<T><<<dim3((unsigned)((film_nr[f] + 255) / 256), 3), dim3(256), 0, s>>>(A, f);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_hfield2(const AdjParams<T> &A, hipStream_t s) {
    k_adj_hfield2<T><<<slot_grid(A.p.n), dim3(64, 4), 0, s>>>(A);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_loss_h(const AdjParams<T> &A, const int *film_cb, hipStream_t s) {
    const long long nr = (long long)(film_cb[3] + 1) * (film_cb[4] + 1) * (film_cb[5] + 1);
    if (nr > 0) k_adj_loss_h<T><<<dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, s>>>(A);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_estep_fused(const AdjParams<T> &A, hipStream_t s) {
    k_adj_efield<T><<<slot_grid(A.p.n), dim3(64, 4), 0, s>>>(A);
    return hipGetLastError();
}

// a[q] += v on the stream (one thread)
template <typename T>
__global__ void __launch_bounds__(64) k_add_one(T *a, long long q, double v) {
    if (threadIdx.x == 0) a[q] += (T)v;
}

template <typename T>
hipError_t launch_add_one(T *a, long long q, double v, hipStream_t s) {
    k_add_one<T><<<dim3(1), dim3(64), 0, s>>>(a, q, v);
    return hipGetLastError();
}

hipError_t launch_copy_segs(const CopySeg *segs, int nseg, int nblk, hipStream_t s) {
    if (nseg == 0) return hipSuccess;
    k_copy_segs<<<dim3(nblk, nseg), dim3(256), 0, s>>>(segs);
    return hipGetLastError();
}

#define MPX_ADJ(T)                                                                              \
    template hipError_t launch_adj_half<T>(const AdjParams<T> &, int, hipStream_t);            \
    template hipError_t launch_adj_estep<T>(const AdjParams<T> &, hipStream_t);                \
    template hipError_t launch_adj_loss<T>(const AdjParams<T> &, int, double, hipStream_t);    \
    template hipError_t launch_adj_eps<T>(const AdjParams<T> &, const int *, double *, hipStream_t);      \
    template hipError_t launch_film_energy<T>(const KParams<T> &, int, double *, double *, double, hipStream_t); \
    template hipError_t launch_adj_half_fused<T>(const AdjParams<T> &, int, int, const long long *, hipStream_t); \
    template hipError_t launch_adj_estep_fused<T>(const AdjParams<T> &, hipStream_t);                           \
    template hipError_t launch_adj_film_part<T>(const AdjParams<T> &, int, const long long *, hipStream_t);     \
    template hipError_t launch_adj_hfield2<T>(const AdjParams<T> &, hipStream_t);                               \
    template hipError_t launch_adj_loss_h<T>(const AdjParams<T> &, const int *, hipStream_t);                    \
    template hipError_t launch_add_one<T>(T *, long long, double, hipStream_t);                                 \
    template hipError_t launch_tape_loss<T>(const KParams<T> &, int, int, double *, hipStream_t, const int *);   \
    template hipError_t launch_adj_loss_tape<T>(const AdjParams<T> &, int, double, const double *,              \
                                                const long long *, int, long long, hipStream_t, const int *);   \
    template hipError_t launch_tape_box<T>(const KParams<T> &, const int *, double *, hipStream_t);             \
    template hipError_t launch_adj_loss_eps_tape<T>(const KParams<T> &, int, double, const double *,             \
                                                    const long long *, int, long long, double *, hipStream_t,    \
                                                    const int *);                                                \
    template hipError_t launch_adj_loss_eps_state<T>(const KParams<T> &, int, double, double *, hipStream_t,     \
                                                     const int *);                                               \
    template hipError_t launch_adj_eps_box<T>(const KParams<T> &, const int *, const double *, const double *,   \
                                              double *, hipStream_t);
MPX_ADJ(float)
MPX_ADJ(double)

} // namespace mpx
