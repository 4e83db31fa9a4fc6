// sweep.hip -- the register-blocked step pass (default schedule): the E full
// step on every non-PEC edge and the merged pair of H/M half steps on every
// non-magnetic face, in one sweep without LDS staging or block barriers.
//
// Scheme (arXiv:2510.22221, Methods, "Numerical Model"): E <- ca E + cb
// (curl H - J) with ca, cb from the edge's mean eps and sigma (the E update
// that follows eq. iterate_H), then H <- H - dt/(2 mu0) curl E twice with the
// new E (eq. iterate_H with M = 0, the two half steps around an integer time).
//
// Layout and schedule:
//   * a block of 64 x 4 threads owns a 64 x 4 tile of (x, y) columns; each
//     thread marches its column up a z-chunk;
//   * at plane k a thread computes E^{n+1} on its own three edges and, from
//     the same loads, the two edges of its +x neighbour and of its +y
//     neighbour that its faces' curls need (recomputed, not exchanged), then
//     the merged H update of plane k-1, whose +z neighbour E^{n+1}(k) it now
//     holds; plane k-1's H and E^{n+1} stay in registers;
//   * neighbour values come from the caches (the +-1 rows and columns of a
//     tile are the own values of the threads next to it), so HBM sees each
//     array about once per step; there is no LDS staging and no barrier in
//     the march, so waves never wait on each other;
//   * E, H and the E-type CPML psi are read from one buffer set and written
//     to the other (ping-pong): recomputed neighbour edges always see the old
//     values;  H-type psi are updated in place (one owner per face);
//   * the coefficients of an edge come from one byte per slot: the material
//     id when the eight cells around the slot share it (all three edges then
//     take the host-computed table entry), 255 otherwise (mixed edges compute
//     ca, cb from the four cell ids, same operation sequence);
//   * tiles that touch no boundary take a path with no wall logic; tiles are
//     dealt to the 8 XCDs in contiguous runs.
// Built without FP contraction: float64 results are bitwise equal to the
// separate-pass kernels and to the LDS-staged fused pass.
#include "stencil.h"

namespace mpx {

constexpr int SWX = 64, SWY = 4;

// one tile: columns (i0 + tx, j0 + ty), planes [k0, k1) owned, plane k1 the
// halo whose E^{n+1} closes the curls of plane k1 - 1
template <typename T, bool WALL>
__device__ __forceinline__ void sweep_tile(const KParams<T> &p, const CoefLds<T> &L, int i0, int j0, int k0, int k1,
                                           bool tpml, bool tsrc, bool tfilm, long long step) {
    const int i = i0 + (int)threadIdx.x, j = j0 + (int)threadIdx.y;
    const bool inside = i < p.n[0] && j < p.n[1];
    const int px = p.px;
    const long long sz = (long long)p.px * p.n[1];
    // plane bases are block-uniform (scalar registers); offsets within a
    // plane are 32-bit
    const int off = min(i, p.n[0] - 1) + px * min(j, p.n[1] - 1);
    const T dx = p.dT[0], dy = p.dT[1], dz = p.dT[2];
    const T ix = p.invd[0], iy = p.invd[1], iz = p.invd[2];
    const T *Ex = p.E[0], *Ey = p.E[1], *Ez = p.E[2];
    const T *Hx = p.H[0], *Hy = p.H[1], *Hz = p.H[2];

    // raw loads relative to (i, j, kc): direct in interior tiles, folded and
    // zero-filled at the boundaries
    int kc = k0;
    auto ld = [&](const T *a, int di, int dj, int dk) -> T {
        if constexpr (WALL) {
            const int kk = fold(kc + dk, p.n[2], p.per[2]);
            const int ii = fold(i + di, p.n[0], p.per[0]), jj = fold(j + dj, p.n[1], p.per[1]);
            if (kk < 0 || ii < 0 || jj < 0) return T(0);
            return (a + (long long)kk * sz)[ii + px * jj];
        } else {
            return (a + (long long)(kc + dk) * sz)[off + di + px * dj];
        }
    };
    auto lc = [&](int di, int dj) -> int {
        if constexpr (WALL) {
            const int kk = fold(kc, p.n[2], p.per[2]);
            const int ii = fold(i + di, p.n[0], p.per[0]), jj = fold(j + dj, p.n[1], p.per[1]);
            if (kk < 0 || ii < 0 || jj < 0) return kMixed;
            return (p.cls + (long long)kk * sz)[ii + px * jj];
        } else {
            return (p.cls + (long long)kc * sz)[off + di + px * dj];
        }
    };

    // plane k0 - 1: the -z neighbours of the first plane's curls
    T hy_km = ld(Hy, 0, 0, -1), hx_km = ld(Hx, 0, 0, -1);
    T hx_xp_km = ld(Hx, 1, 0, -1), hy_yp_km = ld(Hy, 0, 1, -1);
    // plane k - 1 kept for the H update: old H, E^{n+1} own and of +x, +y
    T hx_p = T(0), hy_p = T(0), hz_p = T(0);
    T ex_p = T(0), ey_p = T(0), ez_p = T(0), ey_xp_p = T(0), ez_xp_p = T(0), ex_yp_p = T(0), ez_yp_p = T(0);

    for (int k = k0; k < k1; k++) {
        kc = k;
        // ---- loads (old buffer set)
        const T hx0 = ld(Hx, 0, 0, 0), hy0 = ld(Hy, 0, 0, 0), hz0 = ld(Hz, 0, 0, 0);
        const T hz_xm = ld(Hz, -1, 0, 0), hy_xm = ld(Hy, -1, 0, 0);
        const T hz_ym = ld(Hz, 0, -1, 0), hx_ym = ld(Hx, 0, -1, 0);
        const T hx_xp = ld(Hx, 1, 0, 0), hy_xp = ld(Hy, 1, 0, 0), hz_xp = ld(Hz, 1, 0, 0);
        const T hx_yp = ld(Hx, 0, 1, 0), hy_yp = ld(Hy, 0, 1, 0), hz_yp = ld(Hz, 0, 1, 0);
        const T hx_xpym = ld(Hx, 1, -1, 0), hy_xmyp = ld(Hy, -1, 1, 0);
        const T ex0 = ld(Ex, 0, 0, 0), ey0 = ld(Ey, 0, 0, 0), ez0 = ld(Ez, 0, 0, 0);
        const T ey_xp0 = ld(Ey, 1, 0, 0), ez_xp0 = ld(Ez, 1, 0, 0);
        const T ex_yp0 = ld(Ex, 0, 1, 0), ez_yp0 = ld(Ez, 0, 1, 0);
        const int c0 = lc(0, 0), c_xp = lc(1, 0), c_yp = lc(0, 1);
        const bool own = inside;

        // ---- E^{n+1} at plane k: own edges, +x neighbour's Ey, Ez, +y's Ex, Ez
        const T ex_o = e_upd<T, 0, WALL>(p, L, i, j, k, c0, ex0, dif(hz0, hz_ym, dy, iy), dif(hy0, hy_km, dz, iz),
                                         tpml, tsrc, step, own);
        const T ey_o = e_upd<T, 1, WALL>(p, L, i, j, k, c0, ey0, dif(hx0, hx_km, dz, iz), dif(hz0, hz_xm, dx, ix),
                                         tpml, tsrc, step, own);
        const T ez_o = e_upd<T, 2, WALL>(p, L, i, j, k, c0, ez0, dif(hy0, hy_xm, dx, ix), dif(hx0, hx_ym, dy, iy),
                                         tpml, tsrc, step, own);
        const T ey_xp = e_upd<T, 1, WALL>(p, L, i + 1, j, k, c_xp, ey_xp0, dif(hx_xp, hx_xp_km, dz, iz),
                                          dif(hz_xp, hz0, dx, ix), tpml, tsrc, step, false);
        const T ez_xp = e_upd<T, 2, WALL>(p, L, i + 1, j, k, c_xp, ez_xp0, dif(hy_xp, hy0, dx, ix),
                                          dif(hx_xp, hx_xpym, dy, iy), tpml, tsrc, step, false);
        const T ex_yp = e_upd<T, 0, WALL>(p, L, i, j + 1, k, c_yp, ex_yp0, dif(hz_yp, hz0, dy, iy),
                                          dif(hy_yp, hy_yp_km, dz, iz), tpml, tsrc, step, false);
        const T ez_yp = e_upd<T, 2, WALL>(p, L, i, j + 1, k, c_yp, ez_yp0, dif(hy_yp, hy_xmyp, dx, ix),
                                          dif(hx_yp, hx0, dy, iy), tpml, tsrc, step, false);
        if (own) {
            (p.Eb[0] + (long long)k * sz)[off] = ex_o;
            (p.Eb[1] + (long long)k * sz)[off] = ey_o;
            (p.Eb[2] + (long long)k * sz)[off] = ez_o;
        }

        // ---- merged H/M half steps of plane k - 1
        if (k > k0 && own) {
            const int idx[3] = {i, j, k - 1};
            const long long pm = (long long)(k - 1) * sz;
            bool mag[3] = {false, false, false};
            if (tfilm) {
                mag[0] = face_is_magnetic(p, 0, idx);
                mag[1] = face_is_magnetic(p, 1, idx);
                mag[2] = face_is_magnetic(p, 2, idx);
            }
            if (!mag[0])
                (p.Hb[0] + pm)[off] = h_upd<T, 0>(p, idx, hx_p, dif(ez_yp_p, ez_p, dy, iy), dif(ey_o, ey_p, dz, iz), tpml);
            if (!mag[1])
                (p.Hb[1] + pm)[off] = h_upd<T, 1>(p, idx, hy_p, dif(ex_o, ex_p, dz, iz), dif(ez_xp_p, ez_p, dx, ix), tpml);
            if (!mag[2])
                (p.Hb[2] + pm)[off] = h_upd<T, 2>(p, idx, hz_p, dif(ey_xp_p, ey_p, dx, ix), dif(ex_yp_p, ex_p, dy, iy), tpml);
        }
        // ---- rotate
        hx_p = hx0;
        hy_p = hy0;
        hz_p = hz0;
        ex_p = ex_o;
        ey_p = ey_o;
        ez_p = ez_o;
        ey_xp_p = ey_xp;
        ez_xp_p = ez_xp;
        ex_yp_p = ex_yp;
        ez_yp_p = ez_yp;
        hy_km = hy0;
        hx_km = hx0;
        hx_xp_km = hx_xp;
        hy_yp_km = hy_yp;
    }

    // ---- halo plane k1: Ex, Ey of E^{n+1}(k1) close the z-curls of plane k1-1
    {
        const int k = k1;
        kc = k;
        T ex_o = T(0), ey_o = T(0);
        bool any = true;
        if constexpr (WALL) any = p.per[2] || k < p.n[2];
        if (any) {
            const T hx0 = ld(Hx, 0, 0, 0), hy0 = ld(Hy, 0, 0, 0), hz0 = ld(Hz, 0, 0, 0);
            const T hz_xm = ld(Hz, -1, 0, 0), hz_ym = ld(Hz, 0, -1, 0);
            const T ex0 = ld(Ex, 0, 0, 0), ey0 = ld(Ey, 0, 0, 0);
            const int c0 = lc(0, 0);
            ex_o = e_upd<T, 0, WALL>(p, L, i, j, k, c0, ex0, dif(hz0, hz_ym, dy, iy), dif(hy0, hy_km, dz, iz), tpml,
                                     tsrc, step, false);
            ey_o = e_upd<T, 1, WALL>(p, L, i, j, k, c0, ey0, dif(hx0, hx_km, dz, iz), dif(hz0, hz_xm, dx, ix), tpml,
                                     tsrc, step, false);
        }
        if (inside) {
            const int idx[3] = {i, j, k1 - 1};
            const long long pm = (long long)(k1 - 1) * sz;
            bool mag[3] = {false, false, false};
            if (tfilm) {
                mag[0] = face_is_magnetic(p, 0, idx);
                mag[1] = face_is_magnetic(p, 1, idx);
                mag[2] = face_is_magnetic(p, 2, idx);
            }
            if (!mag[0])
                (p.Hb[0] + pm)[off] = h_upd<T, 0>(p, idx, hx_p, dif(ez_yp_p, ez_p, dy, iy), dif(ey_o, ey_p, dz, iz), tpml);
            if (!mag[1])
                (p.Hb[1] + pm)[off] = h_upd<T, 1>(p, idx, hy_p, dif(ex_o, ex_p, dz, iz), dif(ez_xp_p, ez_p, dx, ix), tpml);
            if (!mag[2])
                (p.Hb[2] + pm)[off] = h_upd<T, 2>(p, idx, hz_p, dif(ey_xp_p, ey_p, dx, ix), dif(ex_yp_p, ex_p, dy, iy), tpml);
        }
    }
}

// tile t of the instance p: block-uniform flags, then the wall or interior
// variant of the march
template <typename T>
__device__ __forceinline__ void sweep_body(const KParams<T> &p, int t, int kchunk) {
    __shared__ CoefLds<T> L;
    stage_coef(p, L, threadIdx.y * SWX + threadIdx.x, SWX * SWY);
    __syncthreads();
    const int nxt = (p.n[0] + SWX - 1) / SWX, nyt = (p.n[1] + SWY - 1) / SWY;
    const int i0 = (t % nxt) * SWX;
    const int j0 = ((t / nxt) % nyt) * SWY;
    const int k0 = (t / (nxt * nyt)) * kchunk;
    const int k1 = min(k0 + kchunk, p.n[2]);
    const long long step = p.step[0];

    // block-uniform flags over the tile with its +-1 halo
    const int lo[3] = {i0 - 1, j0 - 1, k0 - 1}, hi[3] = {i0 + SWX, j0 + SWY, k1};
    bool tpml = false, tsrc = false, tfilm = false;
    for (int a = 0; a < 3; a++) {
        if (p.nlo[a] > 0 && lo[a] < p.nlo[a]) tpml = true;
        if (p.nhi[a] > 0 && hi[a] >= p.n[a] - p.nhi[a]) tpml = true;
    }
    for (int s = 0; s < p.nsrc; s++) {
        const SrcDev &S = p.srcs[s];
        bool in = true;
        for (int a = 0; a < 3; a++)
            if (S.box[a] + S.box[3 + a] <= lo[a] || S.box[a] > hi[a]) in = false;
        if (in) tsrc = true;
    }
    for (int f = 0; f < p.nfilm; f++) {
        const FilmDev &F = p.films[f];
        bool in = true;
        for (int a = 0; a < 3; a++)
            if (F.b0[a] + F.bn[a] <= lo[a] || F.b0[a] > hi[a]) in = false;
        if (in) tfilm = true;
    }
    // a boundary within reach (or a periodic wrap) needs the folded loads
    const bool wall = i0 == 0 || j0 == 0 || k0 == 0 || i0 + SWX >= p.n[0] || j0 + SWY >= p.n[1] || k1 >= p.n[2];
    if (wall) {
        // the periodic wrap brings index 0 next to the far side
        if (p.nsrc && (p.per[0] || p.per[1] || p.per[2])) tsrc = true;
        if (p.nfilm && (p.per[0] || p.per[1] || p.per[2])) tfilm = true;
        sweep_tile<T, true>(p, L, i0, j0, k0, k1, tpml, tsrc, tfilm, step);
    } else {
        sweep_tile<T, false>(p, L, i0, j0, k0, k1, tpml, tsrc, tfilm, step);
    }
}

template <typename T>
__global__ void __launch_bounds__(SWX *SWY) k_sweep(KParams<T> p, int kchunk, int ntile) {
    const int per = (ntile + 7) / 8;
    const int t = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (t >= ntile) return;
    sweep_body<T>(p, t, kchunk);
}

// batched: work[w] = (instance, tile, z-chunk)
template <typename T>
__global__ void __launch_bounds__(SWX *SWY)
    k_sweep_batch(const KParams<T> *__restrict__ plist, const int4 *__restrict__ work, int nwork) {
    const int per = (nwork + 7) / 8;
    const int w = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (w >= nwork) return;
    const int4 wk = work[w];
    sweep_body<T>(plist[wk.x], wk.y, wk.z);
}

// the class byte of every slot: the material id when the (up to) eight
// in-domain cells around the slot, (i-1..i) x (j-1..j) x (k-1..k) folded on
// periodic axes, share it; kMixed otherwise
__global__ void __launch_bounds__(256) k_classify(const uint8_t *__restrict__ id, uint8_t *__restrict__ cls, int nx,
                                                  int ny, int nz, int px, int px_, int py_, int pz_) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    const int k = blockIdx.z;
    if (i >= nx) return;
    int first = -1, same = 1;
    for (int dk = -1; dk <= 0; dk++)
        for (int dj = -1; dj <= 0; dj++)
            for (int di = -1; di <= 0; di++) {
                const int ii = fold(i + di, nx, px_), jj = fold(j + dj, ny, py_), kk = fold(k + dk, nz, pz_);
                if (ii < 0 || jj < 0 || kk < 0) continue;
                const int m = id[(long long)ii + (long long)px * ((long long)jj + (long long)ny * kk)];
                if (first < 0)
                    first = m;
                else if (m != first)
                    same = 0;
            }
    cls[(long long)i + (long long)px * ((long long)j + (long long)ny * k)] = (uint8_t)(same ? first : kMixed);
}

hipError_t launch_classify(const uint8_t *id, uint8_t *cls, const int *n, const int *per, int px, hipStream_t s) {
    hipLaunchKernelGGL(k_classify, dim3((n[0] + 255) / 256, n[1], n[2]), dim3(256), 0, s, id, cls, n[0], n[1], n[2],
                       px, per[0], per[1], per[2]);
    return hipGetLastError();
}

int sweep_tiles(const int *n, int kchunk) {
    return ((n[0] + SWX - 1) / SWX) * ((n[1] + SWY - 1) / SWY) * ((n[2] + kchunk - 1) / kchunk);
}

template <typename T>
hipError_t launch_sweep(const KParams<T> &p, int kchunk, hipStream_t s) {
    const int ntile = sweep_tiles(p.n, kchunk);
    const int nblk = (ntile + 7) / 8 * 8;
    k_sweep<T><<<dim3(nblk), dim3(SWX, SWY), 0, s>>>(p, kchunk, ntile);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sweep_batch(const KParams<T> *plist, const int4 *work, int nwork, hipStream_t s) {
    const int nblk = (nwork + 7) / 8 * 8;
    k_sweep_batch<T><<<dim3(nblk), dim3(SWX, SWY), 0, s>>>(plist, work, nwork);
    return hipGetLastError();
}

template hipError_t launch_sweep<float>(const KParams<float> &, int, hipStream_t);
template hipError_t launch_sweep<double>(const KParams<double> &, int, hipStream_t);
template hipError_t launch_sweep_batch<float>(const KParams<float> *, const int4 *, int, hipStream_t);
template hipError_t launch_sweep_batch<double>(const KParams<double> *, const int4 *, int, hipStream_t);

} // namespace mpx
