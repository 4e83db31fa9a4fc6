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
// boundary use folded, zero-filled loads.  Per-tile CPML / source / film
// flags come from a host table (one per tile shape); edge coefficients come
// from the packed row of the slot's class (its six values in one or two
// 16-byte loads; no per-block staging).
#include "film.h"
#include "stencil.h"

namespace mpx {

constexpr int PTX = kPassTX, PTY = kPassTY;
constexpr int kRsrcWord3 = 0x00020000; // raw buffer resource, gfx9 family

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, long long bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, kRsrcWord3);
}

// AUX: the load's cache-policy bits (2: non-temporal)
template <typename T, int AUX = 0>
__device__ __forceinline__ T bld(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, AUX));
    else
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, AUX));
}

constexpr int kOOB = 0x7ffffff0; // a byte offset past every resource: the load returns 0

// ---------------------------------------------------------------------------
// E pass: E_c <- ca E_c + cb ((curl H)_c - J_c) on the three edges of slot
// (i, j, k); reads H at the slot and at its -x, -y, -z neighbours.  One path
// for every tile: a -1 neighbour wraps on a periodic axis and is, at a wall,
// any in-range value (only edges held at zero would read it); lanes past the
// domain (partial tiles) compute nothing that is stored.  Each edge takes its
// coefficients from the table entry of its slot's class and component (a
// material, or a compound class of a slot whose eight cells differ); on a
// grid with more distinct triples than the class byte holds (XC) the slot's
// 16-bit class also reaches the extended table's rows.  A slot on the mixed
// list (class byte 255, or 16-bit class 0xffff) is skipped and updated
// afterwards by the mixed-slot kernel from the same old values.
// ---------------------------------------------------------------------------
// whether this wave takes the CPML path: a wide tile that reaches CPML slabs
// only along x (flag 1 without 8) needs it only in the waves whose 64 slots,
// with the one-slot halo, reach an x slab (the same test as the tile's, on
// the wave's range; uniform over the wave, so the other waves skip it)
template <typename T, int TX>
__device__ __forceinline__ bool wave_pml(const KParams<T> &p, int bx, int f) {
    if (!(f & 1)) return false;
    if (TX != kWideTX || (f & 8)) return true;
    const int w0 = bx * TX + (__builtin_amdgcn_readfirstlane((int)threadIdx.x) & ~63);
    return (p.nlo[0] > 0 && w0 - 1 < p.nlo[0]) || (p.nhi[0] > 0 && w0 + 64 >= p.n[0] - p.nhi[0]);
}

// CLS: the slot class read, 0 the class byte, 1 the 16-bit class (a grid
// with extended triples), 2 whichever the instance has (batch members of one
// launch differ; the test is uniform over a member's lanes).  f: the tile's
// flag byte, first used after every field load has been issued (so that the
// loads do not wait for it).
template <typename T, int CLS, int TX>
__device__ __forceinline__ void epass_tile(const KParams<T> &p, int i0, int j0, int k, int f, int bxt) {
    const int i = i0 + (int)threadIdx.x, j = j0 + (int)threadIdx.y;
    const bool inside = i < p.n[0] && j < p.n[1];
    const int ic = min(i, p.n[0] - 1), jc = min(j, p.n[1] - 1);
    const long long sz = (long long)p.px * p.n[1];
    const long long pb = sz * (long long)sizeof(T);
    const int es = (int)sizeof(T), rowb = p.px * es;
    const int o = ic + p.px * jc, vo = o * es;
    const int vxm = ic > 0 ? vo - es : (p.per[0] ? vo + (p.n[0] - 1) * es : vo);
    const int vym = jc > 0 ? vo - rowb : (p.per[1] ? vo + (p.n[1] - 1) * rowb : vo);
    const int kb = k > 0 ? k - 1 : (p.per[2] ? p.n[2] - 1 : k);
    const auto rx = make_rsrc(p.H[0] + k * sz, pb), ry = make_rsrc(p.H[1] + k * sz, pb),
               rz = make_rsrc(p.H[2] + k * sz, pb);
    const auto bx = make_rsrc(p.H[0] + kb * sz, pb), by = make_rsrc(p.H[1] + kb * sz, pb);
    // the -z plane's H is read here for the last time (the tiles of its own
    // plane and of the next row read it before): non-temporal
    const T hx0 = bld<T>(rx, vo, 0), hx_km = bld<T, 2>(bx, vo, 0), hx_ym = bld<T>(rx, vym, 0);
    const T hy0 = bld<T>(ry, vo, 0), hy_km = bld<T, 2>(by, vo, 0), hy_xm = bld<T>(ry, vxm, 0);
    const T hz0 = bld<T>(rz, vo, 0), hz_xm = bld<T>(rz, vxm, 0), hz_ym = bld<T>(rz, vym, 0);
    // E, the class and the new E are touched once per pass: non-temporal, so
    // that they leave L2 first and the H rows and planes the neighbouring
    // tiles read again, and the coefficient rows, stay
    T *ex = p.E[0] + k * sz, *ey = p.E[1] + k * sz, *ez = p.E[2] + k * sz;
    const T e0 = __builtin_nontemporal_load(ex + o), e1 = __builtin_nontemporal_load(ey + o),
            e2 = __builtin_nontemporal_load(ez + o);
    // the coefficient triple's row: the class byte (255: the slot is on the
    // mixed list), or with extended triples the 16-bit class (0xffff: on the
    // mixed list), whose rows past 255 are the extended table's
    bool c16 = CLS == 1;
    if constexpr (CLS == 2) c16 = p.cls16 != nullptr;
    int c0;
    if constexpr (CLS == 0)
        c0 = __builtin_nontemporal_load(p.cls + k * sz + o);
    else if constexpr (CLS == 1)
        c0 = __builtin_nontemporal_load(p.cls16 + k * sz + o);
    else if (c16)
        c0 = (p.cls16 + k * sz)[o];
    else
        c0 = (p.cls + k * sz)[o];
    const int kSkip = c16 ? 0xffff : kMixed;
    // the slot's six coefficients in one or two wide loads (a skipped slot
    // reads row 0 and uses none)
    const CoefRow<T> L = coef_row<T>(p.coefv, c0 == kSkip ? 0 : c0);
    const bool tpml = wave_pml<T, TX>(p, bxt, f), tsrc = (f & 2) != 0;
    const long long step = tsrc ? p.step[0] : 0;
    const T dx = p.dT[0], dy = p.dT[1], dz = p.dT[2], ix = p.invd[0], iy = p.invd[1], iz = p.invd[2];
    int q0[3], q1[3], q2[3];
    const bool v0 = inside && e_site<T, 0, true>(p, i, j, k, q0), v1 = inside && e_site<T, 1, true>(p, i, j, k, q1),
               v2 = inside && e_site<T, 2, true>(p, i, j, k, q2);
    if constexpr (sizeof(T) == 8) {
        // float64: the CPML state of one edge at a time (each thread alone
        // reads and writes its edges' psi and E), which keeps the kernel's
        // registers, and with them its occupancy, near the bulk path's
        if (!inside || c0 == kSkip) return;
        T n0 = T(0), n1 = T(0), n2 = T(0);
        {
            Psi2<T> r;
            if (tpml && v0) r = psi_load<T, 0, true>(p, q0);
            if (v0)
                n0 = e_apply<T, 0, CoefRow<T>, false>(p, L, q0, c0, e0, dif(hz0, hz_ym, dy, iy), dif(hy0, hy_km, dz, iz),
                                                     r, tsrc, step);
            if (tpml) psi_store<T, 0>(p.psiE[0], r);
        }
        {
            Psi2<T> r;
            if (tpml && v1) r = psi_load<T, 1, true>(p, q1);
            if (v1)
                n1 = e_apply<T, 1, CoefRow<T>, false>(p, L, q1, c0, e1, dif(hx0, hx_km, dz, iz), dif(hz0, hz_xm, dx, ix),
                                                     r, tsrc, step);
            if (tpml) psi_store<T, 1>(p.psiE[1], r);
        }
        {
            Psi2<T> r;
            if (tpml && v2) r = psi_load<T, 2, true>(p, q2);
            if (v2)
                n2 = e_apply<T, 2, CoefRow<T>, false>(p, L, q2, c0, e2, dif(hy0, hy_xm, dx, ix), dif(hx0, hx_ym, dy, iy),
                                                     r, tsrc, step);
            if (tpml) psi_store<T, 2>(p.psiE[2], r);
        }
        __builtin_nontemporal_store(n0, ex + o);
        __builtin_nontemporal_store(n1, ey + o);
        __builtin_nontemporal_store(n2, ez + o);
        return;
    }
    // float32: every load of the thread before any store (the CPML state of
    // the three edges too)
    Psi2<T> r0, r1, r2;
    if (tpml) {
        if (v0) r0 = psi_load<T, 0, true>(p, q0);
        if (v1) r1 = psi_load<T, 1, true>(p, q1);
        if (v2) r2 = psi_load<T, 2, true>(p, q2);
    }
    if (!inside || c0 == kSkip) return;
    const T n0 = v0 ? e_apply<T, 0, CoefRow<T>, false>(p, L, q0, c0, e0, dif(hz0, hz_ym, dy, iy),
                                                       dif(hy0, hy_km, dz, iz), r0, tsrc, step)
                    : T(0);
    const T n1 = v1 ? e_apply<T, 1, CoefRow<T>, false>(p, L, q1, c0, e1, dif(hx0, hx_km, dz, iz),
                                                       dif(hz0, hz_xm, dx, ix), r1, tsrc, step)
                    : T(0);
    const T n2 = v2 ? e_apply<T, 2, CoefRow<T>, false>(p, L, q2, c0, e2, dif(hy0, hy_xm, dx, ix),
                                                       dif(hx0, hx_ym, dy, iy), r2, tsrc, step)
                    : T(0);
    __builtin_nontemporal_store(n0, ex + o);
    __builtin_nontemporal_store(n1, ey + o);
    __builtin_nontemporal_store(n2, ez + o);
    if (tpml) {
        psi_store<T, 0>(p.psiE[0], r0);
        psi_store<T, 1>(p.psiE[1], r1);
        psi_store<T, 2>(p.psiE[2], r2);
    }
}

// the flag byte of tile (bx, by, k) of the TX x TY table, read through the
// scalar cache (the aligned word that holds it; the tables are whole words):
// a vector load here would put the field loads behind its wait, since the
// vector memory counter completes in order
template <typename T, int TX, int TY>
__device__ __forceinline__ int tile_flag(const KParams<T> &p, int bx, int by, int k) {
    const int nxt = (p.n[0] + TX - 1) / TX, nyt = (p.n[1] + TY - 1) / TY;
    typedef __attribute__((address_space(4))) const uint32_t cword;
    const long long ti = bx + (long long)nxt * (by + (long long)nyt * k);
    const uint32_t w = ((cword *)(TX == PTX ? p.pflags : p.pflags_w))[ti >> 2];
    return (int)((w >> (8 * (int)(ti & 3))) & 0xffu);
}

// a block: the TX x TY slots (bx, by) of plane k, flags from the table of
// that tile shape
template <typename T, int CLS, int TX = PTX, int TY = PTY>
__device__ __forceinline__ void epass_block(const KParams<T> &p, int bx, int by, int k) {
    epass_tile<T, CLS, TX>(p, bx * TX, by * TY, k, tile_flag<T, TX, TY>(p, bx, by, k), bx);
}

// the mixed slots, one thread each: the general path (folded loads; edge
// coefficients from the slot's entry of the extended table, or else from the
// four cell ids), in place after the E pass
template <typename T, bool MIXED>
__device__ __forceinline__ void emixed_apply(const KParams<T> &p, const CoefMem<T> &L, int4 s, int cls) {
    const int i = s.x, j = s.y, k = s.z;
    const T hx0 = ldz(p, p.H[0], i, j, k), hx_km = ldz(p, p.H[0], i, j, k - 1), hx_ym = ldz(p, p.H[0], i, j - 1, k);
    const T hy0 = ldz(p, p.H[1], i, j, k), hy_km = ldz(p, p.H[1], i, j, k - 1), hy_xm = ldz(p, p.H[1], i - 1, j, k);
    const T hz0 = ldz(p, p.H[2], i, j, k), hz_xm = ldz(p, p.H[2], i - 1, j, k), hz_ym = ldz(p, p.H[2], i, j - 1, k);
    const long long q = p.slot(i, j, k);
    const bool tpml = true, tsrc = p.nsrc > 0;
    const long long step = tsrc ? p.step[0] : 0;
    const T dx = p.dT[0], dy = p.dT[1], dz = p.dT[2], ix = p.invd[0], iy = p.invd[1], iz = p.invd[2];
    const T e0 = p.E[0][q], e1 = p.E[1][q], e2 = p.E[2][q];
    const T n0 = e_upd<T, 0, true, true, CoefMem<T>, MIXED>(p, L, i, j, k, cls, e0, dif(hz0, hz_ym, dy, iy),
                                                          dif(hy0, hy_km, dz, iz), tpml, tsrc, step, true);
    const T n1 = e_upd<T, 1, true, true, CoefMem<T>, MIXED>(p, L, i, j, k, cls, e1, dif(hx0, hx_km, dz, iz),
                                                          dif(hz0, hz_xm, dx, ix), tpml, tsrc, step, true);
    const T n2 = e_upd<T, 2, true, true, CoefMem<T>, MIXED>(p, L, i, j, k, cls, e2, dif(hy0, hy_xm, dx, ix),
                                                          dif(hx0, hx_ym, dy, iy), tpml, tsrc, step, true);
    p.E[0][q] = n0;
    p.E[1][q] = n1;
    p.E[2][q] = n2;
}

template <typename T>
__device__ __forceinline__ void emixed_slot(const KParams<T> &p, int m) {
    const int4 s = p.mixed[m];
    if (s.w >= 0)
        emixed_apply<T, false>(p, CoefMem<T>{p.coefx}, s, s.w);
    else
        emixed_apply<T, true>(p, CoefMem<T>{p.coef}, s, kMixed);
}

// ---------------------------------------------------------------------------
// H/M pass: NHALF half steps of the non-magnetic faces of slot (i, j, k);
// reads E at the slot and at its +x, +y, +z neighbours.  A +1 neighbour wraps
// on a periodic axis and reads zero at a wall (the E there is tangential to
// it); lanes past the domain store nothing.
// ---------------------------------------------------------------------------
template <typename T, int NHALF, int TX>
__device__ __forceinline__ void hpass_tile(const KParams<T> &p, int i0, int j0, int k, int f, int bxt) {
    const int i = i0 + (int)threadIdx.x, j = j0 + (int)threadIdx.y;
    const bool inside = i < p.n[0] && j < p.n[1];
    const int ic = min(i, p.n[0] - 1), jc = min(j, p.n[1] - 1);
    const long long sz = (long long)p.px * p.n[1];
    const long long pb = sz * (long long)sizeof(T);
    const int es = (int)sizeof(T), rowb = p.px * es;
    const int o = ic + p.px * jc, vo = o * es;
    const int vxp = ic + 1 < p.n[0] ? vo + es : (p.per[0] ? vo - (p.n[0] - 1) * es : kOOB);
    const int vyp = jc + 1 < p.n[1] ? vo + rowb : (p.per[1] ? vo - (p.n[1] - 1) * rowb : kOOB);
    const int ka = k + 1 < p.n[2] ? k + 1 : (p.per[2] ? 0 : -1);
    const auto rx = make_rsrc(p.E[0] + k * sz, pb), ry = make_rsrc(p.E[1] + k * sz, pb),
               rz = make_rsrc(p.E[2] + k * sz, pb);
    // the plane above; none (every load zero) above a wall
    const auto ax = make_rsrc(p.E[0] + (ka < 0 ? 0 : ka) * sz, ka < 0 ? 0 : pb),
               ay = make_rsrc(p.E[1] + (ka < 0 ? 0 : ka) * sz, ka < 0 ? 0 : pb);
    const auto gx = make_rsrc(p.H[0] + k * sz, pb), gy = make_rsrc(p.H[1] + k * sz, pb),
               gz = make_rsrc(p.H[2] + k * sz, pb);
    const T ex0 = bld<T>(rx, vo, 0), ex_yp = bld<T>(rx, vyp, 0), ex_kp = bld<T>(ax, vo, 0);
    const T ey0 = bld<T>(ry, vo, 0), ey_xp = bld<T>(ry, vxp, 0), ey_kp = bld<T>(ay, vo, 0);
    const T ez0 = bld<T>(rz, vo, 0), ez_xp = bld<T>(rz, vxp, 0), ez_yp = bld<T>(rz, vyp, 0);
    // H and the new H are touched once per pass: non-temporal (the E halo
    // stays in L2); the CPML state keeps the default policy (an x slab's rows
    // share lines with the next row's block)
    const T h0 = bld<T, 2>(gx, vo, 0), h1 = bld<T, 2>(gy, vo, 0), h2 = bld<T, 2>(gz, vo, 0);
    // the tile's flags, first used after every field load has been issued
    const bool tpml = wave_pml<T, TX>(p, bxt, f), tfilm = (f & 4) != 0;
    const T dx = p.dT[0], dy = p.dT[1], dz = p.dT[2], ix = p.invd[0], iy = p.invd[1], iz = p.invd[2];
    const int idx[3] = {ic, jc, k};
    Psi2<T> r0, r1, r2;
    if constexpr (sizeof(T) == 4) {
        if (tpml && inside) {
            r0 = psi_load<T, 0, false>(p, idx);
            r1 = psi_load<T, 1, false>(p, idx);
            r2 = psi_load<T, 2, false>(p, idx);
        }
    }
    bool mag[3] = {false, false, false};
    if (tfilm && inside) {
        mag[0] = face_is_magnetic(p, 0, idx);
        mag[1] = face_is_magnetic(p, 1, idx);
        mag[2] = face_is_magnetic(p, 2, idx);
    }
    if (!inside) return;
    if constexpr (sizeof(T) == 8) {
        // float64: the CPML state of one face at a time (as in the E pass)
        T *hx = p.H[0] + k * sz, *hy = p.H[1] + k * sz, *hz = p.H[2] + k * sz;
        {
            Psi2<T> r;
            if (tpml) r = psi_load<T, 0, false>(p, idx);
            const T n = h_apply<T, 0, NHALF>(p, h0, dif(ez_yp, ez0, dy, iy), dif(ey_kp, ey0, dz, iz), r);
            if (!mag[0]) {
                __builtin_nontemporal_store(n, hx + o);
                if (tpml) psi_store<T, 0>(p.psiH[0], r);
            }
        }
        {
            Psi2<T> r;
            if (tpml) r = psi_load<T, 1, false>(p, idx);
            const T n = h_apply<T, 1, NHALF>(p, h1, dif(ex_kp, ex0, dz, iz), dif(ez_xp, ez0, dx, ix), r);
            if (!mag[1]) {
                __builtin_nontemporal_store(n, hy + o);
                if (tpml) psi_store<T, 1>(p.psiH[1], r);
            }
        }
        {
            Psi2<T> r;
            if (tpml) r = psi_load<T, 2, false>(p, idx);
            const T n = h_apply<T, 2, NHALF>(p, h2, dif(ey_xp, ey0, dx, ix), dif(ex_yp, ex0, dy, iy), r);
            if (!mag[2]) {
                __builtin_nontemporal_store(n, hz + o);
                if (tpml) psi_store<T, 2>(p.psiH[2], r);
            }
        }
        return;
    }
    const T n0 = h_apply<T, 0, NHALF>(p, h0, dif(ez_yp, ez0, dy, iy), dif(ey_kp, ey0, dz, iz), r0);
    const T n1 = h_apply<T, 1, NHALF>(p, h1, dif(ex_kp, ex0, dz, iz), dif(ez_xp, ez0, dx, ix), r1);
    const T n2 = h_apply<T, 2, NHALF>(p, h2, dif(ey_xp, ey0, dx, ix), dif(ex_yp, ex0, dy, iy), r2);
    T *hx = p.H[0] + k * sz, *hy = p.H[1] + k * sz, *hz = p.H[2] + k * sz;
    if (!mag[0]) __builtin_nontemporal_store(n0, hx + o);
    if (!mag[1]) __builtin_nontemporal_store(n1, hy + o);
    if (!mag[2]) __builtin_nontemporal_store(n2, hz + o);
    if (tpml) {
        if (!mag[0]) psi_store<T, 0>(p.psiH[0], r0);
        if (!mag[1]) psi_store<T, 1>(p.psiH[1], r1);
        if (!mag[2]) psi_store<T, 2>(p.psiH[2], r2);
    }
}

template <typename T, int NHALF, int TX = PTX, int TY = PTY>
__device__ __forceinline__ void hpass_block(const KParams<T> &p, int bx, int by, int k) {
    hpass_tile<T, NHALF, TX>(p, bx * TX, by * TY, k, tile_flag<T, TX, TY>(p, bx, by, k), bx);
}

// grid (x tiles, y tiles, planes) in natural order: the blocks resident at
// one time cover a few consecutive planes, so neighbour rows and planes are
// cache hits, and no block decodes its tile with divisions.  Tiles of 64 x 4
// slots, or on grids at least two wide tiles across, 256 x 1 (each block
// then reads and writes 256 consecutive slots of every array: measured 5 %
// (float32) and 9 % (float64) faster per step on a 512-wide grid, slower on
// narrow ones).  In float32 the E pass is held to 72 VGPRs (7 waves per
// SIMD): with the slot's packed coefficient row loaded at once it fits
// without spilling, and it measured 4 % faster than the per-edge table loads
// at 64 VGPRs (at 64 the row spills).  XC: the variant for grids with
// extended-table slots (16-bit classes).
template <typename T, int TX, int TY, bool XC>
__global__ void __launch_bounds__(TX *TY) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 7 : 1, 8)))
k_epass(KParams<T> p) {
    epass_block<T, XC ? 1 : 0, TX, TY>(p, blockIdx.x, blockIdx.y, blockIdx.z);
}

template <typename T, int NHALF, int TX, int TY>
__global__ void __launch_bounds__(TX *TY) k_hbulk(KParams<T> p, int inc_step) {
    if (inc_step && blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x == 0 && threadIdx.y == 0)
        p.step[0] = p.step[0] + 1;
    hpass_block<T, NHALF, TX, TY>(p, blockIdx.x, blockIdx.y, blockIdx.z);
}

// the merged H/M pass and the film kernel's second half step in one launch
// (256 x 1 tiles): the first zf planes of the grid are the film blocks,
// dispatched first so that the latency-bound LLG solves overlap the bulk
// planes.  The two touch disjoint data: the film blocks read the prepass the
// first half step wrote and write M and H of magnetic faces, which the bulk
// blocks load but never store or use.
// the probes of an integer time when every one of them reads only E or the
// film's mean-M partials (which this launch does not write), in the block
// right after the film blocks: its first wavefront reads the step counter,
// samples each probe due and then advances the counter (no other block of
// the launch reads it)
template <typename T>
__device__ __forceinline__ void probe_block(const KParams<T> &p, int nprobe, int inc_step) {
    if (threadIdx.x >= 64) return; // one wavefront does it all
    const long long step = p.step[0];
    for (int pb = 0; pb < nprobe; pb++) {
        const ProbeDev &P = p.probes[pb];
        long long sample;
        if (!probe_due(P, step, sample)) continue; // uniform over the wavefront
        double v[3] = {0.0, 0.0, 0.0};
        probe_e_or_m_values(p, P, v);
        probe_store(p, P, sample, v);
    }
    // lane 0 advances the counter after every lane has read it (one
    // wavefront: its reads above precede this store)
    if (inc_step && threadIdx.x == 0) p.step[0] = step + 1;
}

template <typename T>
__global__ void __launch_bounds__(kWideTX) k_hbulk_film(KParams<T> p, int inc_step, int zf, int nfb, int nprobe) {
    if ((int)blockIdx.z < zf) {
        const int fb = (int)(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z));
        if (fb < nfb)
            film_body(p, 2, 0, fb);
        else if (fb == nfb && nprobe > 0)
            probe_block(p, nprobe, inc_step);
        return;
    }
    const int k = (int)blockIdx.z - zf;
    if (inc_step && nprobe == 0 && blockIdx.x == 0 && blockIdx.y == 0 && k == 0 && threadIdx.x == 0)
        p.step[0] = p.step[0] + 1;
    hpass_block<T, 2, kWideTX, kWideTY>(p, blockIdx.x, blockIdx.y, k);
}

template <typename T>
__global__ void __launch_bounds__(256) k_emixed(KParams<T> p) {
    const int m = blockIdx.x * 256 + threadIdx.x;
    if (m < p.nmixed) emixed_slot<T>(p, m);
}

// batched: work[w] = (instance, x tile, y tile, plane)
template <typename T, bool XC>
__global__ void __launch_bounds__(PTX *PTY)
    k_epass_batch(const KParams<T> *__restrict__ plist, const int4 *__restrict__ work, int nwork) {
    const int w = blockIdx.x;
    if (w >= nwork) return;
    const int4 wk = work[w];
    epass_block<T, XC ? 2 : 0>(plist[wk.x], wk.y, wk.z, wk.w);
}

// work[w] = (instance, first list entry of a 256-entry block)
template <typename T>
__global__ void __launch_bounds__(256)
    k_emixed_batch(const KParams<T> *__restrict__ plist, const int2 *__restrict__ work, int nwork) {
    const int w = blockIdx.x;
    if (w >= nwork) return;
    const int2 wk = work[w];
    const KParams<T> &p = plist[wk.x];
    const int m = wk.y + threadIdx.x;
    if (m < p.nmixed) emixed_slot<T>(p, m);
}

// the step counter of each instance moves with its first block (inc_step)
template <typename T, int NHALF>
__global__ void __launch_bounds__(PTX *PTY)
    k_hbulk_batch(const KParams<T> *__restrict__ plist, const int4 *__restrict__ work, int nwork, int inc_step) {
    const int w = blockIdx.x;
    if (w >= nwork) return;
    const int4 wk = work[w];
    const KParams<T> &p = plist[wk.x];
    if (inc_step && wk.y == 0 && wk.z == 0 && wk.w == 0 && threadIdx.x == 0 && threadIdx.y == 0)
        p.step[0] = p.step[0] + 1;
    hpass_block<T, NHALF>(p, wk.y, wk.z, wk.w);
}

int pass_tiles(const int *n) { return ((n[0] + PTX - 1) / PTX) * ((n[1] + PTY - 1) / PTY) * n[2]; }

template <int TX, int TY>
static dim3 pass_grid(const int *n) {
    return dim3((n[0] + TX - 1) / TX, (n[1] + TY - 1) / TY, n[2]);
}

// the E pass and then its mixed slots
template <typename T>
hipError_t launch_epass(const KParams<T> &p, hipStream_t s) {
    const dim3 gw = pass_grid<kWideTX, kWideTY>(p.n), gn = pass_grid<PTX, PTY>(p.n);
    if (p.wide && p.cls16)
        k_epass<T, kWideTX, kWideTY, true><<<gw, dim3(kWideTX, kWideTY), 0, s>>>(p);
    else if (p.wide)
        k_epass<T, kWideTX, kWideTY, false><<<gw, dim3(kWideTX, kWideTY), 0, s>>>(p);
    else if (p.cls16)
        k_epass<T, PTX, PTY, true><<<gn, dim3(PTX, PTY), 0, s>>>(p);
    else
        k_epass<T, PTX, PTY, false><<<gn, dim3(PTX, PTY), 0, s>>>(p);
    if (p.nmixed > 0) k_emixed<T><<<dim3((p.nmixed + 255) / 256), dim3(256), 0, s>>>(p);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_hbulk(const KParams<T> &p, int nhalf, int inc, hipStream_t s) {
    if (p.wide) {
        const dim3 g = pass_grid<kWideTX, kWideTY>(p.n), b(kWideTX, kWideTY);
        if (nhalf == 1)
            k_hbulk<T, 1, kWideTX, kWideTY><<<g, b, 0, s>>>(p, inc);
        else
            k_hbulk<T, 2, kWideTX, kWideTY><<<g, b, 0, s>>>(p, inc);
    } else {
        const dim3 g = pass_grid<PTX, PTY>(p.n), b(PTX, PTY);
        if (nhalf == 1)
            k_hbulk<T, 1, PTX, PTY><<<g, b, 0, s>>>(p, inc);
        else
            k_hbulk<T, 2, PTX, PTY><<<g, b, 0, s>>>(p, inc);
    }
    return hipGetLastError();
}

// the film's second half step (nblk blocks) and the merged H/M pass; on
// 256 x 1 tiles one launch, else two
template <typename T>
hipError_t launch_hbulk_film(const KParams<T> &p, int nblk, int inc, hipStream_t s, int nprobe) {
    // probes ride in the launch only beside film blocks on 256 x 1 tiles
    if (nprobe > 0 && (nblk == 0 || !p.wide)) return hipErrorInvalidValue;
    if (nblk == 0) return launch_hbulk<T>(p, 2, inc, s);
    if (!p.wide) {
        hipError_t e = launch_film<T>(p, nblk, 2, 0, s);
        if (e != hipSuccess) return e;
        return launch_hbulk<T>(p, 2, inc, s);
    }
    static_assert(kWideTX == 256 && kWideTY == 1, "film blocks are 256 threads along x");
    const dim3 g = pass_grid<kWideTX, kWideTY>(p.n);
    const int per_plane = (int)(g.x * g.y);
    const int zf = (nblk + (nprobe > 0 ? 1 : 0) + per_plane - 1) / per_plane;
    k_hbulk_film<T><<<dim3(g.x, g.y, g.z + zf), dim3(kWideTX, kWideTY), 0, s>>>(p, inc, zf, nblk, nprobe);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_epass_batch(const KParams<T> *plist, const int4 *work, int nwork, const int2 *mwork, int nmwork,
                              bool xcls, hipStream_t s) {
    if (nwork == 0) return hipSuccess;
    if (xcls)
        k_epass_batch<T, true><<<dim3(nwork), dim3(PTX, PTY), 0, s>>>(plist, work, nwork);
    else
        k_epass_batch<T, false><<<dim3(nwork), dim3(PTX, PTY), 0, s>>>(plist, work, nwork);
    if (nmwork > 0) k_emixed_batch<T><<<dim3(nmwork), dim3(256), 0, s>>>(plist, mwork, nmwork);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_hbulk_batch(const KParams<T> *plist, const int4 *work, int nwork, int nhalf, int inc,
                              hipStream_t s) {
    if (nwork == 0) return hipSuccess;
    const dim3 g(nwork), b(PTX, PTY);
    if (nhalf == 1)
        k_hbulk_batch<T, 1><<<g, b, 0, s>>>(plist, work, nwork, inc);
    else
        k_hbulk_batch<T, 2><<<g, b, 0, s>>>(plist, work, nwork, inc);
    return hipGetLastError();
}

#define MPX_PASSES(T)                                                                                      \
    template hipError_t launch_epass<T>(const KParams<T> &, hipStream_t);                                 \
    template hipError_t launch_hbulk<T>(const KParams<T> &, int, int, hipStream_t);                       \
    template hipError_t launch_hbulk_film<T>(const KParams<T> &, int, int, hipStream_t, int);                  \
    template hipError_t launch_epass_batch<T>(const KParams<T> *, const int4 *, int, const int2 *, int,   \
                                              bool, hipStream_t);                                         \
    template hipError_t launch_hbulk_batch<T>(const KParams<T> *, const int4 *, int, int, int, hipStream_t);
MPX_PASSES(float)
MPX_PASSES(double)

} // namespace mpx
