// fused.hip -- the fused step pass: the E full step on every non-PEC edge and
// the merged pair of H/M half steps on every non-magnetic face, in one sweep.
//
// Scheme (arXiv:2510.22221, Methods, "Numerical Model"): E <- ca E + cb
// (curl H - J) with ca, cb from the edge's mean eps and sigma (the E update
// that follows eq. iterate_H), then H <- H - dt/(2 mu0) curl E twice with the
// new E (eq. iterate_H with M = 0, the two half steps around an integer time).
//
// Layout and schedule:
//   * blocks of 64 x 4 threads own a 64 x 8 tile of (x, y) columns, two rows
//     per thread, and march up a z-chunk;
//   * per plane k the block stages H(k) and the material ids of plane k in
//     LDS with a one-cell halo on the low x/y sides and one extra column/row on
//     the high sides, then computes E^{n+1}(k) on its columns (kept in
//     registers) and on the high-side halo, then the merged H update of plane
//     k-1 (whose +z neighbour E^{n+1}(k) it now holds), then publishes
//     E^{n+1}(k) in LDS for the next plane;
//   * E, H and the E-type CPML psi are read from one buffer set and written
//     to the other (ping-pong), so recomputed halo edges never see updated
//     neighbours; H-type psi are updated in place (one owner per face);
//   * tiles are dealt to the 8 XCDs in contiguous runs (blocks go round-robin
//     to XCDs, so block b takes tile (b mod 8) * ceil(ntile/8) + b/8): tiles
//     that share halos share an L2;
//   * block-uniform flags skip the CPML, source and film tests in tiles that
//     have none; edges whose four cells share one id take ca, cb from an LDS
//     table computed on the host with the same operation sequence.
// Every value is evaluated with the operation sequence of the plain
// definition (built without FP contraction), so float64 results are bitwise
// equal to the separate-pass kernels.
#include "device_common.h"

namespace mpx {

constexpr int FTX = 64, FTY = 8;
constexpr int HX_ = FTX + 2, HY_ = FTY + 2;    // staged H / id tile
constexpr int EX_ = FTX + 1, EY_ = FTY + 1;    // E^{n+1} tile (high halo)
constexpr int NHALO = EX_ + FTY;               // high-side halo edge points

template <typename T>
struct FusedLds {
    T h[2][3][HY_][HX_];
    T e[3][EY_][EX_];
    uint8_t id[2][HY_][HX_];
    T ca[256], cb[256];
    uint8_t pec[256];
};

template <int A, int B, int C3>
struct Off { static constexpr int x = A, y = B, z = C3; };

// E^{n+1} of component C at tile point (ii, jj) (0..FTX, 0..FTY), plane k
template <typename T, int C>
__device__ __forceinline__ T fused_e(const KParams<T> &p, const FusedLds<T> &L, int cur, int prv, int i0, int j0,
                                     int ii, int jj, int k, bool tpml, bool tsrc, long long step, bool write,
                                     bool pre = false, T eold_pre = T(0)) {
    constexpr int C1 = (C + 1) % 3, C2 = (C + 2) % 3;
    const int gi = i0 + ii, gj = j0 + jj;
    if (gi > p.n[0] || gj > p.n[1] || k > p.n[2]) return T(0);
    const int raw[3] = {gi, gj, k};
    // walls: tangential edges of a non-periodic face are zero; the high face
    // (index N) of a non-periodic axis is not stored
#pragma unroll
    for (int a = 0; a < 3; a++) {
        if (p.per[a]) continue;
        if (a != C && raw[a] == 0) return T(0);
        if (raw[a] >= p.n[a]) return T(0);
    }
    const int idx[3] = {gi == p.n[0] ? 0 : gi, gj == p.n[1] ? 0 : gj, k == p.n[2] ? 0 : k};
    // the four cells sharing the edge, in the order (C1, C2) offsets
    // (-1,-1), (-1,0), (0,-1), (0,0)
    auto cid = [&](int u, int v) -> int {
        int o[3] = {0, 0, 0};
        o[C1] = u;
        o[C2] = v;
        return L.id[o[2] < 0 ? prv : cur][jj + 1 + o[1]][ii + 1 + o[0]];
    };
    const int m0 = cid(-1, -1), m1 = cid(-1, 0), m2 = cid(0, -1), m3 = cid(0, 0);
    T ca, cb;
    if (m0 == m1 && m0 == m2 && m0 == m3) {
        if (L.pec[m0]) return T(0);
        ca = L.ca[m0];
        cb = L.cb[m0];
    } else {
        const MatDev &A0 = p.mat[m0], &A1 = p.mat[m1], &A2 = p.mat[m2], &A3 = p.mat[m3];
        if (A0.is_pec || A1.is_pec || A2.is_pec || A3.is_pec) return T(0);
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
            const double eps = p.eps0 * (se / 4);
            const double sig = ss / 4;
            const double den = sig / 2.0 + eps / p.dt;
            ca = -(sig / 2.0 - eps / p.dt) / den;
            cb = 1.0 / den;
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
            const double eps = p.eps0 * (se / 4);
            const double sig = ss / 4;
            const double den = sig / 2.0 + eps / p.dt;
            ca = (float)(-(sig / 2.0 - eps / p.dt) / den);
            cb = (float)(1.0 / den);
        }
    }
    // curl H, backward differences; the LDS H tile is offset by one in x, y
    auto hv = [&](int cc, int dx, int dy, int dz) -> T { return L.h[dz < 0 ? prv : cur][cc][jj + 1 + dy][ii + 1 + dx]; };
    int o1[3] = {0, 0, 0}, o2[3] = {0, 0, 0};
    o1[C1] = -1;
    o2[C2] = -1;
    T d1 = dif(hv(C2, 0, 0, 0), hv(C2, o1[0], o1[1], o1[2]), p.dT[C1], p.invd[C1]);
    T d2 = dif(hv(C1, 0, 0, 0), hv(C1, o2[0], o2[1], o2[2]), p.dT[C2], p.invd[C2]);
    if (tpml) {
        const int a1 = idx[C1], a2 = idx[C2];
        if (p.psiE[C][C1] && (a1 < p.nlo[C1] || a1 >= p.n[C1] - p.nhi[C1])) {
            const long long qq = p.psi_index(C1, idx);
            const T ps = p.bE[C1][a1] * p.psiE[C][C1][qq] + p.cE[C1][a1] * d1;
            if (write) p.psiEb[C][C1][qq] = ps;
            d1 += ps;
        }
        if (p.psiE[C][C2] && (a2 < p.nlo[C2] || a2 >= p.n[C2] - p.nhi[C2])) {
            const long long qq = p.psi_index(C2, idx);
            const T ps = p.bE[C2][a2] * p.psiE[C][C2][qq] + p.cE[C2][a2] * d2;
            if (write) p.psiEb[C][C2][qq] = ps;
            d2 += ps;
        }
    }
    double J = 0.0;
    if (tsrc) {
        for (int s = 0; s < p.nsrc; s++) {
            const SrcDev &S = p.src[s];
            if (S.comp != C) continue;
            if (idx[0] < S.box[0] || idx[0] >= S.box[0] + S.box[3] || idx[1] < S.box[1] ||
                idx[1] >= S.box[1] + S.box[4] || idx[2] < S.box[2] || idx[2] >= S.box[2] + S.box[5])
                continue;
            if (step < S.n) J += S.table[step];
        }
    }
    const T eold = pre ? eold_pre : p.E[C][p.slot(idx[0], idx[1], idx[2])];
    return ca * eold + cb * ((d1 - d2) - T(J));
}

template <typename T>
__device__ __forceinline__ T fused_e_any(int c, const KParams<T> &p, const FusedLds<T> &L, int cur, int prv, int i0,
                                         int j0, int ii, int jj, int k, bool tpml, bool tsrc, long long step) {
    if (c == 0) return fused_e<T, 0>(p, L, cur, prv, i0, j0, ii, jj, k, tpml, tsrc, step, false);
    if (c == 1) return fused_e<T, 1>(p, L, cur, prv, i0, j0, ii, jj, k, tpml, tsrc, step, false);
    return fused_e<T, 2>(p, L, cur, prv, i0, j0, ii, jj, k, tpml, tsrc, step, false);
}

// merged pair of H/M half steps for component C at (i, j, km) of an owned
// column; e_{C2}(+C1) etc. come from the published E^{n+1}(km) tile and, for
// +z, from the thread's own E^{n+1}(km+1)
template <typename T, int C>
__device__ __forceinline__ T fused_h(const KParams<T> &p, const FusedLds<T> &L, int tx, int ty, const T *eup,
                                     const int *idx, T h, bool tpml) {
    constexpr int C1 = (C + 1) % 3, C2 = (C + 2) % 3;
    auto ev = [&](int cc, int a) -> T {
        if (a == 2) return eup[cc];
        if (a == 0) return L.e[cc][ty][tx + 1];
        return L.e[cc][ty + 1][tx];
    };
    const T d1r = dif(ev(C2, C1), L.e[C2][ty][tx], p.dT[C1], p.invd[C1]);
    const T d2r = dif(ev(C1, C2), L.e[C1][ty][tx], p.dT[C2], p.invd[C2]);
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
    for (int hs = 0; hs < 2; hs++) {
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


// FROWS rows per thread (blockDim = 64 x 8/FROWS); MINW: minimum waves per
// SIMD the register allocation must allow
template <typename T, int FROWS>
__device__ __forceinline__ void fused_body(const KParams<T> &p, int t, int kchunk) {
    constexpr int FBY = FTY / FROWS;
    constexpr int FNT = FTX * FBY;
    constexpr int NSTAGE = (HY_ * HX_ + FNT - 1) / FNT; // staged points per thread
    __shared__ FusedLds<T> L;
    const int nxt = (p.n[0] + FTX - 1) / FTX, nyt = (p.n[1] + FTY - 1) / FTY;
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int tid = ty * FTX + tx;
    const int i0 = (t % nxt) * FTX;
    const int j0 = ((t / nxt) % nyt) * FTY;
    const int k0 = (t / (nxt * nyt)) * kchunk;
    const int k1 = min(k0 + kchunk, p.n[2]);
    const long long step = p.step[0];

    // block-uniform flags: does the tile (with its halo) touch a CPML slab,
    // a source box, a film's face box?
    bool tpml = false, tsrc = false, tfilm = false;
    {
        const int lo[3] = {i0 - 1, j0 - 1, k0 - 1}, hi[3] = {i0 + FTX, j0 + FTY, k1};
        for (int a = 0; a < 3; a++)
            if (p.nlo[a] > lo[a] + 0 && p.nlo[a] > 0) tpml = true;
        for (int a = 0; a < 3; a++)
            if (p.nhi[a] > 0 && hi[a] >= p.n[a] - p.nhi[a]) tpml = true;
        for (int s = 0; s < p.nsrc; s++) {
            const SrcDev &S = p.src[s];
            bool in = true;
            for (int a = 0; a < 3; a++)
                if (S.box[a] + S.box[3 + a] <= lo[a] + 1 || S.box[a] > hi[a]) in = false;
            if (in) tsrc = true;
        }
        for (int f = 0; f < p.nfilm; f++) {
            const FilmDev &F = p.films[f];
            bool in = true;
            for (int a = 0; a < 3; a++)
                if (F.b0[a] + F.bn[a] <= lo[a] + 1 || F.b0[a] > hi[a]) in = false;
            if (in) tfilm = true;
        }
        // periodic wrap of the high halo brings index 0 into the tile
        if (p.nsrc && (p.per[0] || p.per[1] || p.per[2])) tsrc = true;
        if (p.nfilm && (p.per[0] || p.per[1] || p.per[2])) tfilm = true;
    }

    // coefficient table of single-id edges (a material's three entries are equal)
    for (int q = tid; q < 256; q += FNT) {
        const CoefDev<T> cf = p.coef[kCoefPerClass * q];
        L.ca[q] = cf.ca;
        L.cb[q] = cf.cb;
        L.pec[q] = (uint8_t)cf.pec;
    }

    // staging is split in a fetch into registers (issued one plane ahead, so
    // the loads are in flight while the current plane is computed) and a
    // commit into LDS
    T ph[NSTAGE][3];
    uint8_t pid[NSTAGE];
    T pe[FROWS][3];          // E^n of the owned columns, one plane ahead
    auto fetch = [&](int k) {
        const int kk = fold(k, p.n[2], p.per[2]);
#pragma unroll
        for (int r = 0; r < NSTAGE; r++) {
            const int q = tid + r * FNT;
            ph[r][0] = ph[r][1] = ph[r][2] = T(0);
            pid[r] = 0;
            if (q < HY_ * HX_) {
                const int jj = q / HX_, ii = q % HX_;
                const int gi = fold(i0 - 1 + ii, p.n[0], p.per[0]), gj = fold(j0 - 1 + jj, p.n[1], p.per[1]);
                if (gi >= 0 && gj >= 0 && kk >= 0) {
                    const long long sl = p.slot(gi, gj, kk);
                    ph[r][0] = p.H[0][sl];
                    ph[r][1] = p.H[1][sl];
                    ph[r][2] = p.H[2][sl];
                    pid[r] = p.id[sl];
                }
            }
        }
#pragma unroll
        for (int r = 0; r < FROWS; r++) {
            const int i = i0 + tx, j = j0 + ty + r * FBY;
            pe[r][0] = pe[r][1] = pe[r][2] = T(0);
            if (i < p.n[0] && j < p.n[1] && k >= 0 && k < p.n[2]) {
                const long long q = p.slot(i, j, k);
                pe[r][0] = p.E[0][q];
                pe[r][1] = p.E[1][q];
                pe[r][2] = p.E[2][q];
            }
        }
    };
    auto commit = [&](int buf) {
#pragma unroll
        for (int r = 0; r < NSTAGE; r++) {
            const int q = tid + r * FNT;
            if (q < HY_ * HX_) {
                const int jj = q / HX_, ii = q % HX_;
                L.h[buf][0][jj][ii] = ph[r][0];
                L.h[buf][1][jj][ii] = ph[r][1];
                L.h[buf][2][jj][ii] = ph[r][2];
                L.id[buf][jj][ii] = pid[r];
            }
        }
    };

    fetch(k0 - 1);
    commit((k0 + 1) & 1);
    fetch(k0);
    T hprev[FROWS][3];
    for (int r = 0; r < FROWS; r++)
        for (int c = 0; c < 3; c++) hprev[r][c] = T(0);

    for (int k = k0; k <= k1; k++) {
        const int cur = k & 1, prv = (k + 1) & 1;
        const bool halo_plane = (k == k1);
        commit(cur);
        T eold[FROWS][3];
#pragma unroll
        for (int r = 0; r < FROWS; r++)
            for (int c = 0; c < 3; c++) eold[r][c] = pe[r][c];
        if (k < k1) fetch(k + 1);
        __syncthreads();
        // E^{n+1}(k) on the owned columns (registers) ...
        T eo[FROWS][3];
#pragma unroll
        for (int r = 0; r < FROWS; r++) {
            const int jj = ty + r * FBY;
            const bool inside = (i0 + tx) < p.n[0] && (j0 + jj) < p.n[1] && k < p.n[2];
            const bool own = inside && !halo_plane;
            eo[r][0] = fused_e<T, 0>(p, L, cur, prv, i0, j0, tx, jj, k, tpml, tsrc, step, own, inside, eold[r][0]);
            eo[r][1] = fused_e<T, 1>(p, L, cur, prv, i0, j0, tx, jj, k, tpml, tsrc, step, own, inside, eold[r][1]);
            eo[r][2] = fused_e<T, 2>(p, L, cur, prv, i0, j0, tx, jj, k, tpml, tsrc, step, own, inside, eold[r][2]);
        }
        // ... and on the high-side halo, one component per thread
        T eh = T(0);
        int hq = -1;
        static_assert(3 * NHALO <= 256, "halo items must fit one pass");
        if (tid < 3 * NHALO) {
            hq = tid; // component-major, so most waves take a single component
            const int pt = hq % NHALO, c = hq / NHALO;
            const int ii = pt < EX_ ? pt : FTX;
            const int jj = pt < EX_ ? FTY : pt - EX_;
            eh = fused_e_any<T>(c, p, L, cur, prv, i0, j0, ii, jj, k, tpml, tsrc, step);
        }
        // merged H/M half steps of plane k-1 on the owned columns
        if (k > k0) {
            const int km = k - 1;
#pragma unroll
            for (int r = 0; r < FROWS; r++) {
                const int jj = ty + r * FBY;
                const int i = i0 + tx, j = j0 + jj;
                if (i >= p.n[0] || j >= p.n[1]) continue;
                const int idx[3] = {i, j, km};
                const long long q = p.slot(i, j, km);
                const T eup[3] = {eo[r][0], eo[r][1], eo[r][2]};
                // LDS tile rows of this thread's row r
                const int tyr = jj;
                bool mag[3] = {false, false, false};
                if (tfilm) {
                    mag[0] = face_is_magnetic(p, 0, idx);
                    mag[1] = face_is_magnetic(p, 1, idx);
                    mag[2] = face_is_magnetic(p, 2, idx);
                }
                if (!mag[0]) p.Hb[0][q] = fused_h<T, 0>(p, L, tx, tyr, eup, idx, hprev[r][0], tpml);
                if (!mag[1]) p.Hb[1][q] = fused_h<T, 1>(p, L, tx, tyr, eup, idx, hprev[r][1], tpml);
                if (!mag[2]) p.Hb[2][q] = fused_h<T, 2>(p, L, tx, tyr, eup, idx, hprev[r][2], tpml);
            }
        }
        __syncthreads();
        // publish E^{n+1}(k) for the next plane; write the owned columns
#pragma unroll
        for (int r = 0; r < FROWS; r++) {
            const int jj = ty + r * FBY;
            L.e[0][jj][tx] = eo[r][0];
            L.e[1][jj][tx] = eo[r][1];
            L.e[2][jj][tx] = eo[r][2];
            const int i = i0 + tx, j = j0 + jj;
            if (!halo_plane && i < p.n[0] && j < p.n[1]) {
                const long long q = p.slot(i, j, k);
                p.Eb[0][q] = eo[r][0];
                p.Eb[1][q] = eo[r][1];
                p.Eb[2][q] = eo[r][2];
            }
            hprev[r][0] = L.h[cur][0][jj + 1][tx + 1];
            hprev[r][1] = L.h[cur][1][jj + 1][tx + 1];
            hprev[r][2] = L.h[cur][2][jj + 1][tx + 1];
        }
        if (hq >= 0) {
            const int pt = hq % NHALO, c = hq / NHALO;
            const int ii = pt < EX_ ? pt : FTX;
            const int jj = pt < EX_ ? FTY : pt - EX_;
            L.e[c][jj][ii] = eh;
        }
    }
}

template <typename T, int FROWS, int MINW>
__global__ void __launch_bounds__(FTX *(FTY / FROWS), MINW)
    k_fused(KParams<T> p, int kchunk, int nxt, int nyt, int ntile) {
    // XCD-aware order: blocks are dealt round-robin to the 8 XCDs; give each
    // XCD a contiguous run of tiles
    const int per = (ntile + 7) / 8;
    const int t = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (t >= ntile) return;
    (void)nxt;
    (void)nyt;
    fused_body<T, FROWS>(p, t, kchunk);
}

// batched: work[w] = (instance, tile, z-chunk); the instances' parameters in
// device memory; the same XCD-aware dealing over the whole work list
template <typename T, int FROWS, int MINW>
__global__ void __launch_bounds__(FTX *(FTY / FROWS), MINW)
    k_fused_batch(const KParams<T> *__restrict__ plist, const int4 *__restrict__ work, int nwork) {
    const int per = (nwork + 7) / 8;
    const int w = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (w >= nwork) return;
    const int4 wk = work[w];
    fused_body<T, FROWS>(plist[wk.x], wk.y, wk.z);
}

template <typename T>
hipError_t launch_fused_batch(const KParams<T> *plist, const int4 *work, int nwork, int variant, hipStream_t s) {
    const int nblk = (nwork + 7) / 8 * 8;
    switch (variant) {
    case 2:
        k_fused_batch<T, 2, 4><<<dim3(nblk), dim3(FTX, FTY / 2), 0, s>>>(plist, work, nwork);
        break;
    case 3:
        k_fused_batch<T, 1, 2><<<dim3(nblk), dim3(FTX, FTY), 0, s>>>(plist, work, nwork);
        break;
    case 4:
        k_fused_batch<T, 1, 4><<<dim3(nblk), dim3(FTX, FTY), 0, s>>>(plist, work, nwork);
        break;
    default:
        k_fused_batch<T, 2, 2><<<dim3(nblk), dim3(FTX, FTY / 2), 0, s>>>(plist, work, nwork);
        break;
    }
    return hipGetLastError();
}

template hipError_t launch_fused_batch<float>(const KParams<float> *, const int4 *, int, int, hipStream_t);
template hipError_t launch_fused_batch<double>(const KParams<double> *, const int4 *, int, int, hipStream_t);

// variant: 1 = 2 rows/thread, >= 2 waves/SIMD; 2 = 2 rows, >= 4 waves;
// 3 = 1 row/thread (512 threads), >= 2 waves; 4 = 1 row, >= 4 waves
template <typename T>
hipError_t launch_fused(const KParams<T> &p, int kchunk, int variant, hipStream_t s) {
    const int nxt = (p.n[0] + FTX - 1) / FTX, nyt = (p.n[1] + FTY - 1) / FTY;
    const int nzc = (p.n[2] + kchunk - 1) / kchunk;
    const int ntile = nxt * nyt * nzc;
    const int nblk = (ntile + 7) / 8 * 8;
    switch (variant) {
    case 2:
        k_fused<T, 2, 4><<<dim3(nblk), dim3(FTX, FTY / 2), 0, s>>>(p, kchunk, nxt, nyt, ntile);
        break;
    case 3:
        k_fused<T, 1, 2><<<dim3(nblk), dim3(FTX, FTY), 0, s>>>(p, kchunk, nxt, nyt, ntile);
        break;
    case 4:
        k_fused<T, 1, 4><<<dim3(nblk), dim3(FTX, FTY), 0, s>>>(p, kchunk, nxt, nyt, ntile);
        break;
    default:
        k_fused<T, 2, 2><<<dim3(nblk), dim3(FTX, FTY / 2), 0, s>>>(p, kchunk, nxt, nyt, ntile);
        break;
    }
    return hipGetLastError();
}

template hipError_t launch_fused<float>(const KParams<float> &, int, int, hipStream_t);
template hipError_t launch_fused<double>(const KParams<double> &, int, int, hipStream_t);

} // namespace mpx
