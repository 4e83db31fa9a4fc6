// film.h -- the magnetic-face LLG half step of one block of film sites and
// the float64 helpers it uses; included by the kernel files that launch it
// (the film kernels, and the merged H/M pass that runs the second half step
// of a pair beside the bulk faces).
//
// Scheme: arXiv:2510.22221, Methods, "Numerical Model": B^ = H + M,
// B^* = B^ - dt/(2 mu0) curl E (eq. iterate_H); the trapezoidal LLG (eqs.
// llg_tra4-llg_tra6) at its fixed point, normalised to Ms; H = B^*_c - M_c.
#pragma once

#include "device_common.h"

namespace mpx {

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

__device__ __forceinline__ void cross3(const double *a, const double *b, double *r) {
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}

__device__ __forceinline__ double dot3(const double *a, const double *b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// the site solve of one magnetic face: P, Q are B^* and B^ at the face
// (own family) and the means of the four nearest faces of each other family,
// M the magnetisation of the half step's start; the bias is added to P and Q
// here.  Trapezoidal LLG over the half step at its fixed point:
// b = M - k (M x H_eff(M)) with H_eff = Q - M, a = -(k P + (alpha/Ms) M),
// X = (b + (a.b) a - a x b) / (1 + |a|^2), M' = Ms X / |X|
__device__ __forceinline__ void llg_site(double kf, const double *H0, double ms, double al, double ga, double *P,
                                         double *Q, const double *M, double *Mn) {
    for (int w = 0; w < 3; w++) {
        P[w] += H0[w];
        Q[w] += H0[w];
    }
    const double kk = kf * ga;
    // b = M^n - k (M^n x H_eff^n), with H_eff^n = Q - M^n
    double MxQ[3], b[3], a[3];
    cross3(M, Q, MxQ);
    for (int w = 0; w < 3; w++) b[w] = M[w] - kk * MxQ[w];
    // a at the fixed point: H_eff^{n+1} = P - M^{n+1}
    for (int w = 0; w < 3; w++) a[w] = -(kk * P[w] + (al / ms) * M[w]);
    // X = (b + (a.b) a - a x b) / (1 + |a|^2), then M' = Ms X/|X|
    double axb[3], X[3];
    cross3(a, b, axb);
    const double ab = dot3(a, b), aa = dot3(a, a);
    for (int w = 0; w < 3; w++) X[w] = (b[w] + ab * a[w] - axb[w]) / (1.0 + aa);
    const double nx = sqrt(dot3(X, X));
    for (int w = 0; w < 3; w++) Mn[w] = ms * X[w] / nx;
}

template <typename T>
__device__ __forceinline__ void film_body(const KParams<T> &p, int phase, int inc_step, int blk) {
    __shared__ double red[256];
    if (inc_step && blk == 0 && threadIdx.x == 0) p.step[0] = p.step[0] + 1;
    const int4 bt = block_entry(p.blocktab, blk); // film, family, first local index
    const int f = bt.x, c = bt.y;
    const FilmDev F = film_desc(p.films, f);
    const long long l = (long long)bt.z + threadIdx.x;
    double own = 0.0;
    if (l < F.ns) {
        int idx[3];
        idx[0] = F.b0[0] + (int)(l % F.bn[0]);
        idx[1] = F.b0[1] + (int)((l / F.bn[0]) % F.bn[1]);
        idx[2] = F.b0[2] + (int)(l / ((long long)F.bn[0] * F.bn[1]));
        const double ms = F.prm[(c * 3 + 0) * F.ns + l];
        const double al = F.prm[(c * 3 + 1) * F.ns + l];
        const double ga = F.prm[(c * 3 + 2) * F.ns + l];
        if (ms > 0.0) {
            // index in the grown face box (every face the solve reads lies in it)
            // (-1 outside it: cannot happen for accepted film placements)
            auto ext = [&](const int *q) -> long long {
                const int r0 = q[0] - F.e0[0], r1 = q[1] - F.e0[1], r2 = q[2] - F.e0[2];
                if (r0 < 0 || r0 >= F.en[0] || r1 < 0 || r1 >= F.en[1] || r2 < 0 || r2 >= F.en[2]) return -1;
                return (long long)r0 + (long long)F.en[0] * ((long long)r1 + (long long)F.en[1] * r2);
            };
            const long long le = ext(idx);
            const double *Bn = phase == 1 ? F.Bn : F.Bn2, *Bs = phase == 1 ? F.Bs : F.Bs2;
            const double bn = le >= 0 ? Bn[c * F.nse + le] : 0.0, bs = le >= 0 ? Bs[c * F.nse + le] : 0.0;
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
                        const long long lq = ext(q);
                        vn[u][v] = lq >= 0 ? Bn[cp * F.nse + lq] : 0.0;
                        vs[u][v] = lq >= 0 ? Bs[cp * F.nse + lq] : 0.0;
                    }
                Q[cp] = ((vn[0][0] + vn[1][0]) + (vn[0][1] + vn[1][1])) * 0.25;
                P[cp] = ((vs[0][0] + vs[1][0]) + (vs[0][1] + vs[1][1])) * 0.25;
            }
            const double *Msrc = (phase == 1) ? F.M : F.M1;
            for (int w = 0; w < 3; w++) M[w] = Msrc[(c * 3 + w) * F.ns + l];
            double Mn[3];
            llg_site(p.kf, p.H0, ms, al, ga, P, Q, M, Mn);
            const double hnew = bs - Mn[c];
            if (phase == 1) {
                for (int w = 0; w < 3; w++) F.M1[(c * 3 + w) * F.ns + l] = Mn[w];
                F.H1[c * F.ns + l] = hnew;
                if (F.Bn2 && le >= 0) {
                    // the phase-2 prepass of this face: B^ = H1 + M1_c, B^* =
                    // B^ - dt/(2 mu0) curl E with the same E (the prepass
                    // left that term in this face's B^* slot)
                    const double cu = F.Bs2[c * F.nse + le];
                    const double b2 = hnew + Mn[c];
                    F.Bn2[c * F.nse + le] = b2;
                    F.Bs2[c * F.nse + le] = b2 - cu;
                }
            } else {
                for (int w = 0; w < 3; w++) F.M[(c * 3 + w) * F.ns + l] = Mn[w];
                p.Hw[c][p.slot(idx[0], idx[1], idx[2])] = (T)hnew;
            }
            own = Mn[c];
        }
    }
    // block partial of the own component (mean-M probes, which read it
    // between the two half steps: the second half step's would go unread)
    if (phase != 1) return;
    red[threadIdx.x] = own;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) p.partial[blk] = red[0];
}

} // namespace mpx
