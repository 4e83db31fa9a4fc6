// passes.hip -- the separate-pass schedule: an E pass, then an H/M pass, each
// in place with one thread per slot (blocks of 64 x 4 slots of one plane).
// Also the bracket half steps of every schedule (an H/M pass with one half
// step) and the E pass of a call's last step.
//
// Scheme (arXiv:2510.22221, Methods, "Numerical Model"): the E update that
// follows eq. iterate_H, and eq. iterate_H with M = 0 for non-magnetic faces
// (the magnetic ones are the film kernels' work).
//
// Memory access: in blocks that touch no boundary every load is a raw buffer
// load (a scalar resource per array whose base is the block's lowest plane,
// a 32-bit byte offset per lane, and the neighbour plane as a scalar offset),
// so the address work per load is one or two integer operations; blocks at a
// boundary use folded, zero-filled loads.  Blocks are dealt to the XCDs in
// contiguous runs, so the neighbour rows and the neighbour plane a block
// reads were fetched into the same L2 by the blocks just before it.
#include "stencil.h"

namespace mpx {

constexpr int PTX = 64, PTY = 4;
constexpr int kRsrcWord3 = 0x00020000; // raw buffer resource, gfx9 family

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, long long bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, kRsrcWord3);
}

template <typename T>
__device__ __forceinline__ T bld(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    else
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

// block-uniform flags of a one-plane tile with its +-1 halo: CPML slab,
// source box, film face box within reach
template <typename T>
__device__ __forceinline__ void pass_flags(const KParams<T> &p, int i0, int j0, int k, bool &tpml, bool &tsrc,
                                           bool &tfilm) {
    const int lo[3] = {i0 - 1, j0 - 1, k - 1}, hi[3] = {i0 + PTX, j0 + PTY, k + 1};
    tpml = tsrc = tfilm = false;
#pragma unroll
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
    // a periodic wrap brings index 0 next to the far side
    if (p.per[0] || p.per[1] || p.per[2]) {
        if (p.nsrc) tsrc = true;
        if (p.nfilm) tfilm = true;
    }
}

// ---------------------------------------------------------------------------
// E pass: E_c <- ca E_c + cb ((curl H)_c - J_c) on the three edges of slot
// (i, j, k); reads H at the slot and at its -x, -y, -z neighbours
// ---------------------------------------------------------------------------
template <typename T, bool WALL>
__device__ __forceinline__ void epass_tile(const KParams<T> &p, const CoefLds<T> &L, int i0, int j0, int k, bool tpml,
                                           bool tsrc) {
    const int i = i0 + (int)threadIdx.x, j = j0 + (int)threadIdx.y;
    if (WALL && (i >= p.n[0] || j >= p.n[1])) return;
    const long long sz = (long long)p.px * p.n[1];
    const int o = i + p.px * j;
    T hx0, hy0, hz0, hx_km, hy_km, hz_xm, hy_xm, hz_ym, hx_ym;
    int c0;
    if constexpr (!WALL) {
        const long long base = (long long)(k - 1) * sz;
        const long long nb = 2 * sz * (long long)sizeof(T);
        const int P = (int)(sz * (long long)sizeof(T));
        const int vo = o * (int)sizeof(T), vxm = vo - (int)sizeof(T), vym = vo - p.px * (int)sizeof(T);
        const auto rx = make_rsrc(p.H[0] + base, nb), ry = make_rsrc(p.H[1] + base, nb),
                   rz = make_rsrc(p.H[2] + base, nb);
        hx0 = bld<T>(rx, vo, P);
        hx_km = bld<T>(rx, vo, 0);
        hx_ym = bld<T>(rx, vym, P);
        hy0 = bld<T>(ry, vo, P);
        hy_km = bld<T>(ry, vo, 0);
        hy_xm = bld<T>(ry, vxm, P);
        hz0 = bld<T>(rz, vo, P);
        hz_xm = bld<T>(rz, vxm, P);
        hz_ym = bld<T>(rz, vym, P);
        c0 = (p.cls + (long long)k * sz)[o];
    } else {
        hx0 = ldz(p, p.H[0], i, j, k);
        hx_km = ldz(p, p.H[0], i, j, k - 1);
        hx_ym = ldz(p, p.H[0], i, j - 1, k);
        hy0 = ldz(p, p.H[1], i, j, k);
        hy_km = ldz(p, p.H[1], i, j, k - 1);
        hy_xm = ldz(p, p.H[1], i - 1, j, k);
        hz0 = ldz(p, p.H[2], i, j, k);
        hz_xm = ldz(p, p.H[2], i - 1, j, k);
        hz_ym = ldz(p, p.H[2], i, j - 1, k);
        c0 = (p.cls + (long long)k * sz)[o];
    }
    T *ex = p.E[0] + (long long)k * sz, *ey = p.E[1] + (long long)k * sz, *ez = p.E[2] + (long long)k * sz;
    const long long step = tsrc ? p.step[0] : 0;
    const T dx = p.dT[0], dy = p.dT[1], dz = p.dT[2], ix = p.invd[0], iy = p.invd[1], iz = p.invd[2];
    const T e0 = ex[o], e1 = ey[o], e2 = ez[o];
    ex[o] = e_upd<T, 0, WALL, true>(p, L, i, j, k, c0, e0, dif(hz0, hz_ym, dy, iy), dif(hy0, hy_km, dz, iz), tpml,
                                    tsrc, step, true);
    ey[o] = e_upd<T, 1, WALL, true>(p, L, i, j, k, c0, e1, dif(hx0, hx_km, dz, iz), dif(hz0, hz_xm, dx, ix), tpml,
                                    tsrc, step, true);
    ez[o] = e_upd<T, 2, WALL, true>(p, L, i, j, k, c0, e2, dif(hy0, hy_xm, dx, ix), dif(hx0, hx_ym, dy, iy), tpml,
                                    tsrc, step, true);
}

template <typename T>
__device__ __forceinline__ void epass_body(const KParams<T> &p, int t) {
    __shared__ CoefLds<T> L;
    stage_coef(p, L, threadIdx.y * PTX + threadIdx.x, PTX * PTY);
    __syncthreads();
    const int nxt = (p.n[0] + PTX - 1) / PTX, nyt = (p.n[1] + PTY - 1) / PTY;
    const int i0 = (t % nxt) * PTX, j0 = ((t / nxt) % nyt) * PTY, k = t / (nxt * nyt);
    bool tpml, tsrc, tfilm;
    pass_flags(p, i0, j0, k, tpml, tsrc, tfilm);
    // the E pass reads the -x, -y, -z neighbours
    const bool wall = i0 == 0 || j0 == 0 || k == 0 || i0 + PTX > p.n[0] || j0 + PTY > p.n[1];
    if (wall)
        epass_tile<T, true>(p, L, i0, j0, k, tpml, tsrc);
    else
        epass_tile<T, false>(p, L, i0, j0, k, tpml, tsrc);
}

// ---------------------------------------------------------------------------
// H/M pass: NHALF half steps of the non-magnetic faces of slot (i, j, k);
// reads E at the slot and at its +x, +y, +z neighbours
// ---------------------------------------------------------------------------
template <typename T, int NHALF, bool WALL>
__device__ __forceinline__ void hpass_tile(const KParams<T> &p, int i0, int j0, int k, bool tpml, bool tfilm) {
    const int i = i0 + (int)threadIdx.x, j = j0 + (int)threadIdx.y;
    if (WALL && (i >= p.n[0] || j >= p.n[1])) return;
    const long long sz = (long long)p.px * p.n[1];
    const int o = i + p.px * j;
    T ex0, ey0, ez0, ex_yp, ex_kp, ey_xp, ey_kp, ez_xp, ez_yp;
    if constexpr (!WALL) {
        const long long base = (long long)k * sz;
        const long long nb = 2 * sz * (long long)sizeof(T);
        const int P = (int)(sz * (long long)sizeof(T));
        const int vo = o * (int)sizeof(T), vxp = vo + (int)sizeof(T), vyp = vo + p.px * (int)sizeof(T);
        const auto rx = make_rsrc(p.E[0] + base, nb), ry = make_rsrc(p.E[1] + base, nb),
                   rz = make_rsrc(p.E[2] + base, nb);
        ex0 = bld<T>(rx, vo, 0);
        ex_yp = bld<T>(rx, vyp, 0);
        ex_kp = bld<T>(rx, vo, P);
        ey0 = bld<T>(ry, vo, 0);
        ey_xp = bld<T>(ry, vxp, 0);
        ey_kp = bld<T>(ry, vo, P);
        ez0 = bld<T>(rz, vo, 0);
        ez_xp = bld<T>(rz, vxp, 0);
        ez_yp = bld<T>(rz, vyp, 0);
    } else {
        ex0 = ldz(p, p.E[0], i, j, k);
        ex_yp = ldz(p, p.E[0], i, j + 1, k);
        ex_kp = ldz(p, p.E[0], i, j, k + 1);
        ey0 = ldz(p, p.E[1], i, j, k);
        ey_xp = ldz(p, p.E[1], i + 1, j, k);
        ey_kp = ldz(p, p.E[1], i, j, k + 1);
        ez0 = ldz(p, p.E[2], i, j, k);
        ez_xp = ldz(p, p.E[2], i + 1, j, k);
        ez_yp = ldz(p, p.E[2], i, j + 1, k);
    }
    const T dx = p.dT[0], dy = p.dT[1], dz = p.dT[2], ix = p.invd[0], iy = p.invd[1], iz = p.invd[2];
    T *hx = p.H[0] + (long long)k * sz, *hy = p.H[1] + (long long)k * sz, *hz = p.H[2] + (long long)k * sz;
    const int idx[3] = {i, j, k};
    bool mag[3] = {false, false, false};
    if (tfilm) {
        mag[0] = face_is_magnetic(p, 0, idx);
        mag[1] = face_is_magnetic(p, 1, idx);
        mag[2] = face_is_magnetic(p, 2, idx);
    }
    if (!mag[0]) hx[o] = h_upd<T, 0, NHALF>(p, idx, hx[o], dif(ez_yp, ez0, dy, iy), dif(ey_kp, ey0, dz, iz), tpml);
    if (!mag[1]) hy[o] = h_upd<T, 1, NHALF>(p, idx, hy[o], dif(ex_kp, ex0, dz, iz), dif(ez_xp, ez0, dx, ix), tpml);
    if (!mag[2]) hz[o] = h_upd<T, 2, NHALF>(p, idx, hz[o], dif(ey_xp, ey0, dx, ix), dif(ex_yp, ex0, dy, iy), tpml);
}

template <typename T, int NHALF>
__device__ __forceinline__ void hpass_body(const KParams<T> &p, int t) {
    const int nxt = (p.n[0] + PTX - 1) / PTX, nyt = (p.n[1] + PTY - 1) / PTY;
    const int i0 = (t % nxt) * PTX, j0 = ((t / nxt) % nyt) * PTY, k = t / (nxt * nyt);
    bool tpml, tsrc, tfilm;
    pass_flags(p, i0, j0, k, tpml, tsrc, tfilm);
    // the H pass reads the +x, +y, +z neighbours
    const bool wall = i0 + PTX >= p.n[0] || j0 + PTY >= p.n[1] || k + 1 >= p.n[2];
    if (wall)
        hpass_tile<T, NHALF, true>(p, i0, j0, k, tpml, tfilm);
    else
        hpass_tile<T, NHALF, false>(p, i0, j0, k, tpml, tfilm);
}

__device__ __forceinline__ int xcd_tile(int ntile) {
    const int per = (ntile + 7) / 8;
    return (blockIdx.x % 8) * per + blockIdx.x / 8;
}

template <typename T>
__global__ void __launch_bounds__(PTX *PTY) k_epass(KParams<T> p, int ntile) {
    const int t = xcd_tile(ntile);
    if (t >= ntile) return;
    epass_body<T>(p, t);
}

template <typename T, int NHALF>
__global__ void __launch_bounds__(PTX *PTY) k_hbulk(KParams<T> p, int ntile, int inc_step) {
    if (inc_step && blockIdx.x == 0 && threadIdx.x == 0 && threadIdx.y == 0) p.step[0] = p.step[0] + 1;
    const int t = xcd_tile(ntile);
    if (t >= ntile) return;
    hpass_body<T, NHALF>(p, t);
}

// batched: work[w] = (instance, tile)
template <typename T>
__global__ void __launch_bounds__(PTX *PTY)
    k_epass_batch(const KParams<T> *__restrict__ plist, const int2 *__restrict__ work, int nwork) {
    const int w = xcd_tile(nwork);
    if (w >= nwork) return;
    const int2 wk = work[w];
    epass_body<T>(plist[wk.x], wk.y);
}

// the step counter of each instance moves with its tile 0 (inc_step)
template <typename T, int NHALF>
__global__ void __launch_bounds__(PTX *PTY)
    k_hbulk_batch(const KParams<T> *__restrict__ plist, const int2 *__restrict__ work, int nwork, int inc_step) {
    const int w = xcd_tile(nwork);
    if (w >= nwork) return;
    const int2 wk = work[w];
    const KParams<T> &p = plist[wk.x];
    if (inc_step && wk.y == 0 && threadIdx.x == 0 && threadIdx.y == 0) p.step[0] = p.step[0] + 1;
    hpass_body<T, NHALF>(p, wk.y);
}

int pass_tiles(const int *n) { return ((n[0] + PTX - 1) / PTX) * ((n[1] + PTY - 1) / PTY) * n[2]; }

template <typename T>
hipError_t launch_epass(const KParams<T> &p, hipStream_t s) {
    const int ntile = pass_tiles(p.n);
    k_epass<T><<<dim3((ntile + 7) / 8 * 8), dim3(PTX, PTY), 0, s>>>(p, ntile);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_hbulk(const KParams<T> &p, int nhalf, int inc, hipStream_t s) {
    const int ntile = pass_tiles(p.n);
    const dim3 g((ntile + 7) / 8 * 8), b(PTX, PTY);
    if (nhalf == 1)
        k_hbulk<T, 1><<<g, b, 0, s>>>(p, ntile, inc);
    else
        k_hbulk<T, 2><<<g, b, 0, s>>>(p, ntile, inc);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_epass_batch(const KParams<T> *plist, const int2 *work, int nwork, hipStream_t s) {
    if (nwork == 0) return hipSuccess;
    k_epass_batch<T><<<dim3((nwork + 7) / 8 * 8), dim3(PTX, PTY), 0, s>>>(plist, work, nwork);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_hbulk_batch(const KParams<T> *plist, const int2 *work, int nwork, int nhalf, int inc,
                              hipStream_t s) {
    if (nwork == 0) return hipSuccess;
    const dim3 g((nwork + 7) / 8 * 8), b(PTX, PTY);
    if (nhalf == 1)
        k_hbulk_batch<T, 1><<<g, b, 0, s>>>(plist, work, nwork, inc);
    else
        k_hbulk_batch<T, 2><<<g, b, 0, s>>>(plist, work, nwork, inc);
    return hipGetLastError();
}

#define MPX_PASSES(T)                                                                                      \
    template hipError_t launch_epass<T>(const KParams<T> &, hipStream_t);                                 \
    template hipError_t launch_hbulk<T>(const KParams<T> &, int, int, hipStream_t);                       \
    template hipError_t launch_epass_batch<T>(const KParams<T> *, const int2 *, int, hipStream_t);        \
    template hipError_t launch_hbulk_batch<T>(const KParams<T> *, const int2 *, int, int, int, hipStream_t);
MPX_PASSES(float)
MPX_PASSES(double)

} // namespace mpx
