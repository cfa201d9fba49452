// cosmo.hip -- gfx950 kernels and the C ABI of libcosmo.so (include/cosmo.h).
//
// Launch layout of the distance and adjoint kernels: 256-lane blocks; a block
// owns 256 consecutive redshifts (one per lane, coalesced loads/stores along z)
// and a tile of `ct` consecutive cosmologies that it walks in order, so a shared
// redshift row is loaded once per block and reused across the tile.  The
// per-cosmology record (roots, constants, Jacobian) is block-uniform and is read
// through the scalar cache.  The flat block index is split as
// (cosmology tile, z block) with z blocks fastest.
#include <hip/hip_runtime.h>

#include <atomic>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "../../include/cosmo.h"
#include "adjoint.hpp"
#include "between.hpp"

namespace cosmo {

constexpr int kBlock = 256;

// ---------------------------------------------------------------- kernels
__global__ void k_setup(const double *__restrict__ params, int64_t n, CosmoRec *__restrict__ recs,
                        int32_t *__restrict__ info) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    // built in place: a private record would live in scratch memory (~0.5 KB per lane)
    CosmoRec &r = recs[c];
    setup_cosmo(params + 4 * c, r);
    if (info) info[c] = r.info;
}

__global__ void k_roots(const double *__restrict__ params, int64_t n, double *__restrict__ roots,
                        int32_t *__restrict__ info) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    CosmoRec r;
    setup_cosmo(params + 4 * c, r);
    double *o = roots + 8 * c;
    bool have = !(r.info & COSMO_INFO_DOMAIN);
    const double nan = __builtin_nan("");
    if (have) {
        const LaneConst<double> &d = r.d;
        o[0] = d.r0 - 1.0; o[1] = 0.0;
        o[2] = d.r1re - 1.0; o[3] = d.r1im;
        o[4] = (r.pair ? d.r1re : d.r2) - 1.0; o[5] = r.pair ? -d.r1im : 0.0;
        o[6] = r.rl - 1.0; o[7] = (r.info & COSMO_INFO_QUARTIC) ? 0.0 : nan;
    } else {
        for (int i = 0; i < 8; ++i) o[i] = nan;
    }
    if (info) info[c] = r.info;
}

template <typename T, int KIND, bool PAIR>
__device__ __forceinline__ T eval_kind(const CosmoRec &r, T z, bool &used_gl) {
    const LaneConst<T> &k = lane_of<T>(r);
    used_gl = false;
    if (KIND == COSMO_T) return k.th * t_hat<T, PAIR>(r, z);
    if (KIND == COSMO_X) {
        int route;
        const T v = k.dh * x_hat<T, PAIR>(r, z, route);
        used_gl = route == kXRouteQuad;
        return v;
    }
    T chi = chi_hat<T, PAIR>(k, z);
    T a, b, c, d;
    return observable<T>(KIND, k, chi, z, T(0), a, b, c, d);
}

// Block index -> (cosmology tile, z block).
__device__ __forceinline__ void block_tile(int64_t nzb, int64_t &tile, int64_t &zb) {
    const int64_t b = blockIdx.x;
    tile = b / nzb;
    zb = b - tile * nzb;
}

template <typename T, int KIND>
__global__ __launch_bounds__(kBlock) void k_forward(const CosmoRec *__restrict__ recs, int64_t n_cosmo,
                                                     const T *__restrict__ z, int64_t n_z, int64_t zstride,
                                                     T *__restrict__ out, int32_t *__restrict__ info,
                                                     int ct, int64_t nzb) {
    // grid: x = z block, y = cosmology tile (fewer than 65536 tiles, see tiling)
    const int64_t tile = blockIdx.y, zb = blockIdx.x;
    const int64_t i = zb * kBlock + threadIdx.x;
    const bool active = i < n_z;
    const int64_t c0 = tile * ct;
    const int64_t c1 = c0 + ct < n_cosmo ? c0 + ct : n_cosmo;
    if (!active) return; // no cross-lane work below
    const uint32_t i32 = (uint32_t)i; // n_z < 2^29 (checked on the host)
    auto lane = [&](int64_t c, T zz) __attribute__((always_inline)) {
        const CosmoRec &r = recs[c];
        T v;
        bool used_gl = false;
        if (!r.valid) v = Fp<T>::nan();
        else if (r.pair) v = eval_kind<T, KIND, true>(r, zz, used_gl);
        else v = eval_kind<T, KIND, false>(r, zz, used_gl);
        __builtin_nontemporal_store(v, (out + c * n_z) + i32);
        if (KIND == COSMO_X && info) {
            unsigned long long m = __ballot(used_gl);
            if (m && (int)__lane_id() == __ffsll((long long)m) - 1) atomicOr(info + c, COSMO_INFO_X_QUADRATURE);
        }
    };
    if (zstride == 0) {
        const T zz = z[i];
        // the shared redshift has arrived before the loop starts, so the loop holds no
        // load and no wait for one (a wait on the in-order vector-memory counter would
        // also wait for the previous cosmology's stores)
        __builtin_amdgcn_s_waitcnt(0);
        for (int64_t c = c0; c < c1; ++c) lane(c, zz);
    } else {
        for (int64_t c = c0; c < c1; ++c) lane(c, (z + c * zstride)[i32]);
    }
}

// Route counts (cosmo_route_counts): per lane, the route its value takes (X: x_hat's
// route; the other kinds have one) and whether its adjoint takes the Leibniz quadrature,
// decided by the functions the forward and adjoint kernels branch on; per wave the
// popcounts of their ballots, one 64-bit atomic add per wave and count.
template <typename T, int KIND, bool PAIR>
__device__ __forceinline__ void route_lane(const CosmoRec &r, T z, bool act, unsigned long long *cnt) {
    int vr = kXRouteCarlson;
    if (KIND == COSMO_X && act) (void)x_hat<T, PAIR>(r, z, vr);
    const bool aq = act && adjoint_quadrature_lane<T>(KIND, r, z);
    const unsigned long long n[4] = {(unsigned long long)__popcll(__ballot(act && vr == kXRouteCarlson)),
                                     (unsigned long long)__popcll(__ballot(act && vr == kXRouteFp64)),
                                     (unsigned long long)__popcll(__ballot(act && vr == kXRouteQuad)),
                                     (unsigned long long)__popcll(__ballot(aq))};
    if (__lane_id() == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (n[q]) atomicAdd(cnt + q, n[q]);
    }
}

template <typename T, int KIND>
__global__ __launch_bounds__(kBlock) void k_routes(const CosmoRec *__restrict__ recs, int64_t n_cosmo,
                                                    const T *__restrict__ z, int64_t n_z, int64_t zstride,
                                                    unsigned long long *__restrict__ counts, int ct, int64_t nzb) {
    int64_t tile, zb;
    block_tile(nzb, tile, zb);
    const int64_t i = zb * kBlock + threadIdx.x;
    const bool act = i < n_z;
    const int64_t c0 = tile * ct;
    const int64_t c1 = c0 + ct < n_cosmo ? c0 + ct : n_cosmo;
    for (int64_t c = c0; c < c1; ++c) {
        const CosmoRec &r = recs[c];
        if (!r.valid) continue;
        const T zz = act ? z[c * zstride + i] : T(1);
        if (r.pair) route_lane<T, KIND, true>(r, zz, act, counts + 4 * c);
        else route_lane<T, KIND, false>(r, zz, act, counts + 4 * c);
    }
}

template <typename T> __global__ void k_fill_zero_u64(T *__restrict__ p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = T(0);
}

// Observables between two redshifts (between.hpp): lane i of a cosmology evaluates the
// pair (z1[i], z2[i]); tiling as k_forward (a one-dimensional grid of tile-major blocks).
template <typename T, int KIND>
__global__ __launch_bounds__(kBlock) void k_between(const CosmoRec *__restrict__ recs, int64_t n_cosmo,
                                                     const T *__restrict__ z1, const T *__restrict__ z2,
                                                     int64_t n_z, int64_t zstride, T *__restrict__ out,
                                                     int ct, int64_t nzb) {
    int64_t tile, zb;
    block_tile(nzb, tile, zb);
    const int64_t i = zb * kBlock + threadIdx.x;
    if (i >= n_z) return;
    const int64_t c0 = tile * ct;
    const int64_t c1 = c0 + ct < n_cosmo ? c0 + ct : n_cosmo;
    for (int64_t c = c0; c < c1; ++c) {
        const CosmoRec &r = recs[c];
        const T a = z1[c * zstride + i], bb = z2[c * zstride + i];
        T v;
        if (!r.valid) v = Fp<T>::nan();
        else if (r.pair) v = eval_between<T, KIND, true>(r, a, bb);
        else v = eval_between<T, KIND, false>(r, a, bb);
        out[c * n_z + i] = v;
    }
}

// Accumulator slots of the adjoint (per lane, then per wave, then per cosmology),
// w = cot dout/dbase:
//   0 sum w base, 1 sum w dbase/dsigma, 2 sum w dbase/drho0,
//   3/4 sum w dbase/drho1 (re, im) [pair] or drho1, drho2 [real]   (root-chain lanes),
//   5 sum cot dout/dOk, 6 sum cot dout/dH0,
//   7..9 sum w dbase/d(Om, OL, Or)                                  (quadrature lanes),
//   10   sum -ivar (obs - out)^2 / 2                                (likelihood mode).
constexpr int kAcc = 11;
constexpr int kAccLoss = 10;

// One lane of the adjoint: accumulates the cotangent-weighted partials into acc,
// returns the z-gradient in gz and the observable in val (the quantity
// cosmo_distance evaluates; used_gl flags the quadrature route of X).
// LIKE (Gaussian likelihood): cin is the observed value, the residual res = obs - out
// adds -ivar res^2 / 2 to the loss slot and the cotangent is wc ivar res;
// otherwise cin is the cotangent.
template <typename T, int KIND, bool PAIR, bool LIKE, int ROUTE = 0>
__device__ __forceinline__ void vjp_lane(const CosmoRec &r, T z, T cin, T ivar, T wc, T acc[kAcc], T &gz, T &val,
                                         bool &used_gl) {
    LaneGrad<T> o;
    if (ROUTE == 1) lane_grad_small<T, KIND, PAIR>(r, z, o);
    else lane_grad<T, KIND, PAIR>(r, z, o, used_gl);
    val = o.val;
    T cot = cin;
    if (LIKE) {
        const T res = cin - o.val;
        const T rv = res * ivar;
        acc[kAccLoss] += T(-0.5) * res * rv;
        cot = wc * rv;
    }
    gz = cot * o.dz;
    // increments formed per route, then added to every slot unconditionally (keeps
    // the accumulators in registers)
    T d[5], e[3];
    if (o.quad) {
        const double w = (double)cot * (double)o.s;
#pragma unroll
        for (int i = 0; i < 5; ++i) d[i] = T(0);
#pragma unroll
        for (int i = 0; i < 3; ++i) e[i] = T(w * o.q[i]);
    } else {
        const T w = cot * o.s;
#pragma unroll
        for (int i = 0; i < 5; ++i) d[i] = w * o.p[i];
#pragma unroll
        for (int i = 0; i < 3; ++i) e[i] = T(0);
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) acc[i] += d[i];
    acc[5] += cot * o.dok;
    acc[6] += cot * o.dh;
#pragma unroll
    for (int i = 0; i < 3; ++i) acc[7 + i] += e[i];
}

// Sum over the 64 lanes of a wave (all lanes active), with DPP lane moves instead of
// LDS permutes: quad permutes (lane ^ 1, lane ^ 2) and row rotations by 4 and 8 leave
// every lane with its 16-lane row sum; row broadcast 15 (into rows 1 and 3) and 31
// (into rows 2 and 3) carry the row sums up, so lane 63 holds the total, which is
// returned to every lane.  Lanes a move does not write receive zero.
template <int CTRL, int ROWS> __device__ __forceinline__ uint32_t dpp_move(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xF, false);
}
template <int CTRL, int ROWS> __device__ __forceinline__ float dpp_move(float v) {
    return __builtin_bit_cast(float, dpp_move<CTRL, ROWS>(__builtin_bit_cast(uint32_t, v)));
}
template <int CTRL, int ROWS> __device__ __forceinline__ double dpp_move(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint64_t lo = dpp_move<CTRL, ROWS>((uint32_t)b), hi = dpp_move<CTRL, ROWS>((uint32_t)(b >> 32));
    return __builtin_bit_cast(double, (hi << 32) | lo);
}
__device__ __forceinline__ float lane63(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}
__device__ __forceinline__ double lane63(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, 63);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), 63);
    return __builtin_bit_cast(double, (hi << 32) | lo);
}
template <typename T> __device__ __forceinline__ T wave_sum(T v) {
    v += dpp_move<0xB1, 0xF>(v);  // quad_perm [1,0,3,2]
    v += dpp_move<0x4E, 0xF>(v);  // quad_perm [2,3,0,1]
    v += dpp_move<0x124, 0xF>(v); // row_ror:4
    v += dpp_move<0x128, 0xF>(v); // row_ror:8
    v += dpp_move<0x142, 0xA>(v); // row_bcast:15
    v += dpp_move<0x143, 0xC>(v); // row_bcast:31
    return lane63(v);
}

// Cross-lane moves for wave_sum8: lane ^ X within 32 lanes (swizzle in bit mode:
// and-mask 0x1F, xor-mask X) and any lane (permute by byte address).
template <int X> __device__ __forceinline__ float swap_x(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, v), (X << 10) | 0x1F));
}
template <int X> __device__ __forceinline__ double swap_x(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint64_t lo = (uint32_t)__builtin_amdgcn_ds_swizzle((int)(uint32_t)b, (X << 10) | 0x1F);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_ds_swizzle((int)(uint32_t)(b >> 32), (X << 10) | 0x1F);
    return __builtin_bit_cast(double, (hi << 32) | lo);
}
__device__ __forceinline__ float permute(float v, int addr) {
    return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(addr, __builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double permute(double v, int addr) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint64_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)b);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)(b >> 32));
    return __builtin_bit_cast(double, (hi << 32) | lo);
}

// Wave sums of eight slots at once (all lanes active): a transposed butterfly.  Each
// exchange step pairs the lanes that differ in one bit of the lane index (bit 0, 1, then
// 3: quad permutes and a row rotation by 8, i.e. lane ^ 8 within a 16-lane row); a lane
// keeps the half of its slots that this bit selects and adds the partner's copy of the
// same half.  After three steps a lane holds one slot, j = 4 b0 + 2 b1 + b3, summed over
// eight lanes; the rest is a plain sum over lane bits 2, 4 and 5.  Returns the wave total
// of slot j(lane) on every lane: about a third of the lane operations of eight wave_sum
// calls.
template <typename T> __device__ __forceinline__ T wave_sum8(const T v[8], int lane) {
    const bool h0 = lane & 1, h1 = lane & 2, h3 = lane & 8;
    T a[4], b[2];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const T keep = h0 ? v[j + 4] : v[j], send = h0 ? v[j] : v[j + 4];
        a[j] = keep + dpp_move<0xB1, 0xF>(send);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const T keep = h1 ? a[j + 2] : a[j], send = h1 ? a[j] : a[j + 2];
        b[j] = keep + dpp_move<0x4E, 0xF>(send);
    }
    const T keep = h3 ? b[1] : b[0], send = h3 ? b[0] : b[1];
    T c = keep + dpp_move<0x128, 0xF>(send);
    c += swap_x<4>(c);
    c += swap_x<16>(c);
    c += permute(c, (lane ^ 32) << 2);
    return c;
}

// The wave's partial sums of one cosmology's accumulators into its row of kAcc slots:
// slots 0-6 and the loss by wave_sum8 (its lanes 0-3 and 8-11 store them), the three
// quadrature slots one by one, skipped when no lane of the wave touched them.
template <typename T> __device__ __forceinline__ void store_partials(const T acc[kAcc], T *__restrict__ row, int lane) {
    // the lane masks and offsets below are derived here, once per call (an opaque copy of
    // the lane index keeps the compiler from hoisting them out of the cosmology loop,
    // where they would occupy registers across the lane loops and spill)
    asm volatile("" : "+v"(lane));
    const T v8[8] = {acc[0], acc[1], acc[2], acc[3], acc[4], acc[5], acc[6], acc[kAccLoss]};
    const T tot = wave_sum8(v8, lane);
    if ((lane & 0x34) == 0) {
        const int j = 4 * (lane & 1) + (lane & 2) + ((lane >> 3) & 1);
        row[j == 7 ? kAccLoss : j] = tot;
    }
#pragma unroll
    for (int s = 7; s < 10; ++s) {
        T v = T(0);
        if (__ballot(acc[s] != T(0))) v = wave_sum(acc[s]);
        if (lane == 0) row[s] = v;
    }
}

// Redshifts per lane of the adjoint: lane t of z-block zb handles
// i = zb * kBlock * ZPT + t + k * kBlock, k < ZPT (coalesced for every k).  The
// parameter partials of a cosmology are summed over the lane's ZPT redshifts in
// registers, then over the wave, and each wave writes its own partial (no block
// barrier).  The shared-z gradient is summed over the tile's cosmologies in
// thread-private LDS slots (gzl[k][t]), which keeps the rolled k-loop free of
// dynamically indexed register arrays.  Both partials are stored in the lane
// precision (they are sums in that precision already) and summed in FP64 by
// k_finalize_params and k_reduce_gz.
//
// General loop: every route of lane_grad (near-multiple-root cosmologies, X).
template <typename T, int KIND, bool PAIR, int ZPT, bool LIKE>
__device__ __forceinline__ void vjp_cosmo_general(const CosmoRec &r, int64_t c, const T *__restrict__ z, int64_t n_z,
                                                  int64_t zstride, const T *__restrict__ cot, const T *__restrict__ ivar,
                                                  T wc, int64_t base, T acc[kAcc], T *gzl, T *__restrict__ gz_out,
                                                  T *__restrict__ out, int32_t *__restrict__ info) {
#pragma unroll 1
    for (int k = 0; k < ZPT; ++k) {
        const int64_t i = base + (int64_t)k * kBlock;
        if (i >= n_z) break;
        const T zz = z[c * zstride + i];
        T gz, val;
        bool used_gl = false;
        if (LIKE) vjp_lane<T, KIND, PAIR, true>(r, zz, cot[c * zstride + i], ivar[c * zstride + i], wc, acc, gz, val, used_gl);
        else vjp_lane<T, KIND, PAIR, false>(r, zz, cot[c * n_z + i], T(0), T(0), acc, gz, val, used_gl);
        if (out) {
            out[c * n_z + i] = val;
            if (KIND == COSMO_X && info) {
                unsigned long long m = __ballot(used_gl);
                if (m && (int)__lane_id() == __ffsll((long long)m) - 1) atomicOr(info + c, COSMO_INFO_X_QUADRATURE);
            }
        }
        if (zstride != 0) {
            if (gz_out) gz_out[c * n_z + i] = gz;
        } else {
            gzl[k * kBlock + threadIdx.x] += gz;
        }
    }
}

// Element i of a row through a 32-bit byte offset (a row holds fewer than 2^32 bytes:
// n_z < 2^29, checked on the host), so that an address is the row's scalar base plus one
// vector offset, with no 64-bit address arithmetic per lane.
template <typename T> __device__ __forceinline__ T *row_at(T *row, uint32_t i) {
    return (T *)((char *)row + i * (uint32_t)sizeof(T));
}
template <typename T> __device__ __forceinline__ const T *row_at(const T *row, uint32_t i) {
    return (const T *)((const char *)row + i * (uint32_t)sizeof(T));
}

// The root-chain lanes (lane_grad_root) run in a loop of their own, which touches only
// the slots that route writes (0..6, and the loss); FP32 lanes below kSmallZ32 are
// marked and run afterwards in a second pass that only waves holding such lanes enter
// (the redshifts of a row are typically sorted, so those lanes gather in few waves).
// Near-multiple-root cosmologies (uniform per cosmology) and X take the general loop.
template <typename T, int KIND, bool PAIR, int ZPT, bool LIKE>
__device__ __forceinline__ void vjp_cosmo(const CosmoRec &r, int64_t c, const T *__restrict__ z, int64_t n_z,
                                          int64_t zstride, const T *__restrict__ cot, const T *__restrict__ ivar,
                                          T wc, int64_t base, T acc[kAcc], T *gzl, T *__restrict__ gz_out,
                                          T *__restrict__ out, int32_t *__restrict__ info) {
    constexpr bool fp32 = sizeof(T) == 4;
    if (KIND == COSMO_X || direct_mode(KIND, r, fp32)) {
        vjp_cosmo_general<T, KIND, PAIR, ZPT, LIKE>(r, c, z, n_z, zstride, cot, ivar, wc, base, acc, gzl, gz_out, out,
                                                   info);
        return;
    }
    // row pointers of this cosmology (uniform) and 32-bit lane offsets (n_z < 2^29 is
    // checked on the host): the loads and stores take a scalar base and a vector offset
    const uint32_t i0 = (uint32_t)base, nz = (uint32_t)n_z;
    const T *__restrict__ zr = z + c * zstride;
    const T *__restrict__ cr = LIKE ? cot + c * zstride : cot + c * n_z;
    const T *__restrict__ vr = LIKE ? ivar + c * zstride : nullptr;
    T *__restrict__ orow = out ? out + c * n_z : nullptr;
    T *__restrict__ grow = gz_out ? gz_out + c * n_z : nullptr;
    // FP64: the next redshift's inputs are loaded before this one's outputs are stored
    // (one in-order counter tracks vector loads and stores, so a wait for loads issued
    // after a store would also wait for the store; 4% on the headline FP64 step).  The
    // FP32 loop loads in place: the prefetch's registers cost it more at eight waves.
    constexpr bool pre = sizeof(T) == 8;
    uint32_t deferred = 0;
    T zn = T(0), cn = T(0), vn = T(0);
    if (pre && i0 < nz) {
        zn = *row_at(zr, i0);
        cn = LIKE ? *row_at(cr, i0) : __builtin_nontemporal_load(row_at(cr, i0));
        if (LIKE) vn = *row_at(vr, i0);
    }
#pragma unroll 1
    for (int k = 0; k < ZPT; ++k) {
        const uint32_t i = i0 + (uint32_t)(k * kBlock);
        if (i >= nz) break;
        T zz, cin, vin;
        if (pre) {
            zz = zn; cin = cn; vin = vn;
            const uint32_t i1 = i + kBlock;
            if (k + 1 < ZPT && i1 < nz) {
                zn = *row_at(zr, i1);
                cn = LIKE ? *row_at(cr, i1) : __builtin_nontemporal_load(row_at(cr, i1));
                if (LIKE) vn = *row_at(vr, i1);
            }
        } else {
            zz = *row_at(zr, i);
            cin = LIKE ? *row_at(cr, i) : __builtin_nontemporal_load(row_at(cr, i));
            vin = LIKE ? *row_at(vr, i) : T(0);
        }
        if (small_z_lane<T>(zz)) {
            deferred |= 1u << k;
            continue;
        }
        RootGrad<T> o;
        lane_grad_root<T, KIND, PAIR>(r, zz, o);
        T cv;
        if (LIKE) {
            const T res = cin - o.val;
            const T rv = res * vin;
            acc[kAccLoss] += T(-0.5) * res * rv;
            cv = wc * rv;
        } else {
            cv = cin;
        }
        const T w = cv * o.s, wp = w * o.ps;
        acc[0] += w * o.p[0];
#pragma unroll
        for (int q = 1; q < 5; ++q) acc[q] += wp * o.p[q];
        acc[5] += cv * o.dok;
        acc[6] += cv * o.dh;
        const T gz = cv * o.dz;
        if (orow) __builtin_nontemporal_store(o.val, row_at(orow, i));
        if (zstride != 0) {
            if (grow) *row_at(grow, i) = gz;
        } else {
            gzl[k * kBlock + threadIdx.x] += gz;
        }
    }
    if (fp32 && __ballot(deferred != 0)) {
#pragma unroll 1
        for (int k = 0; k < ZPT; ++k) {
            if (!(deferred & (1u << k))) continue;
            const int64_t i = base + (int64_t)k * kBlock;
            const T zz = z[c * zstride + i];
            T gz, val;
            bool used_gl = false;
            if (LIKE) vjp_lane<T, KIND, PAIR, true, 1>(r, zz, cot[c * zstride + i], ivar[c * zstride + i], wc, acc, gz, val, used_gl);
            else vjp_lane<T, KIND, PAIR, false, 1>(r, zz, cot[c * n_z + i], T(0), T(0), acc, gz, val, used_gl);
            if (out) out[c * n_z + i] = val;
            if (zstride != 0) {
                if (gz_out) gz_out[c * n_z + i] = gz;
            } else {
                gzl[k * kBlock + threadIdx.x] += gz;
            }
        }
    }
}

// Occupancy: the comoving-distance-family adjoint is held to seven waves per SIMD (72
// VGPRs) on the FP32 path (on the headline workload as fast as eight waves at 64 VGPRs
// with the value output and 2-3% faster without it, with fewer spills; six waves at 80
// VGPRs were 3-6% slower) and to 128 VGPRs, four waves, on the FP64 path (its coefficients
// in scalar registers, see kc); T, X and the volume keep the compiler's allocation.
template <typename T, int KIND> constexpr int adjoint_min_waves() {
    return (KIND == COSMO_T || KIND == COSMO_X || KIND == COSMO_VC) ? 1 : (sizeof(T) == 4 ? 7 : 4);
}

template <typename T, int KIND, int ZPT, bool LIKE>
__global__ __launch_bounds__(kBlock, (adjoint_min_waves<T, KIND>())) void k_vjp(const CosmoRec *__restrict__ recs, int64_t n_cosmo,
                                                 const T *__restrict__ z, int64_t n_z, int64_t zstride,
                                                 const T *__restrict__ cot, const T *__restrict__ ivar,
                                                 const double *__restrict__ wcs, T *__restrict__ pacc,
                                                 T *__restrict__ gz_out, T *__restrict__ gz_part,
                                                 T *__restrict__ out, int32_t *__restrict__ info,
                                                 int ct, int64_t nzb) {
    __shared__ T gzl[ZPT * kBlock];
    int64_t tile, zb;
    block_tile(nzb, tile, zb);
    const int64_t base = zb * (int64_t)(kBlock * ZPT) + threadIdx.x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t nwz = nzb * (kBlock / 64);           // wave partials per cosmology
    const int64_t gw = zb * (kBlock / 64) + wave;
    const int64_t c0 = tile * ct;
    const int64_t c1 = c0 + ct < n_cosmo ? c0 + ct : n_cosmo;
    for (int k = 0; k < ZPT; ++k) gzl[k * kBlock + threadIdx.x] = T(0);
    for (int64_t c = c0; c < c1; ++c) {
        const CosmoRec &r = recs[c];
        T acc[kAcc];
#pragma unroll
        for (int s = 0; s < kAcc; ++s) acc[s] = T(0);
        if (r.valid) {
            const T wc = LIKE ? (wcs ? T(wcs[c]) : T(1)) : T(0);
            if (r.pair) vjp_cosmo<T, KIND, true, ZPT, LIKE>(r, c, z, n_z, zstride, cot, ivar, wc, base, acc, gzl, gz_out, out, info);
            else vjp_cosmo<T, KIND, false, ZPT, LIKE>(r, c, z, n_z, zstride, cot, ivar, wc, base, acc, gzl, gz_out, out, info);
        } else {
            for (int k = 0; k < ZPT; ++k) {
                const int64_t i = base + (int64_t)k * kBlock;
                if (i >= n_z) break;
                if (out) out[c * n_z + i] = Fp<T>::nan();
                if (zstride != 0) {
                    if (gz_out) gz_out[c * n_z + i] = Fp<T>::nan();
                } else {
                    gzl[k * kBlock + threadIdx.x] = Fp<T>::nan();
                }
            }
        }
        if (pacc) store_partials(acc, pacc + (c * nwz + gw) * kAcc, lane);
    }
    if (zstride == 0 && gz_out) {
        for (int k = 0; k < ZPT; ++k) {
            const int64_t i = base + (int64_t)k * kBlock;
            if (i >= n_z) break;
            const T v = gzl[k * kBlock + threadIdx.x];
            if (gz_part) gz_part[tile * n_z + i] = v;
            else gz_out[i] = v;
        }
    }
}

// Adjoint of the observables between two redshifts (D_C family and T): the structure of k_vjp
// (ZPT pairs per lane, per-wave partial sums of the same accumulator slots, finalised by
// k_finalize_params) with two redshift gradients; for limits shared by all cosmologies
// the z1- and z2-gradients are summed over the tile in thread-private LDS slots.  CO: the
// cosmology satisfies between_chain_only (no quadrature route on any lane).
template <typename T, int KIND, bool PAIR, int ZPT, bool CO>
__device__ __forceinline__ void between_vjp_cosmo(const CosmoRec &r, int64_t c, const T *__restrict__ z1,
                                                  const T *__restrict__ z2, int64_t n_z, int64_t zstride,
                                                  const T *__restrict__ cot, int64_t base, T acc[kAcc], T *gl1,
                                                  T *gl2, T *__restrict__ g1_out, T *__restrict__ g2_out,
                                                  T *__restrict__ out) {
#pragma unroll 1
    for (int k = 0; k < ZPT; ++k) {
        const int64_t i = base + (int64_t)k * kBlock;
        if (i >= n_z) break;
        const T a = z1[c * zstride + i], b = z2[c * zstride + i];
        const T w = cot[c * n_z + i];
        LaneGrad2<T> o;
        lane_grad_between<T, KIND, PAIR, CO>(r, a, b, o);
        const LaneGrad<T> &g = o.g;
        T d[5], e[3];
        if (!CO && g.quad) {
            const double ws = (double)w * (double)g.s;
#pragma unroll
            for (int q = 0; q < 5; ++q) d[q] = T(0);
#pragma unroll
            for (int q = 0; q < 3; ++q) e[q] = T(ws * g.q[q]);
        } else {
            const T ws = w * g.s;
#pragma unroll
            for (int q = 0; q < 5; ++q) d[q] = ws * g.p[q];
#pragma unroll
            for (int q = 0; q < 3; ++q) e[q] = T(0);
        }
#pragma unroll
        for (int q = 0; q < 5; ++q) acc[q] += d[q];
        if (KIND != COSMO_T) acc[5] += w * g.dok; // the time coordinate has no curvature transform
        acc[6] += w * g.dh;
        if (!CO) {
#pragma unroll
            for (int q = 0; q < 3; ++q) acc[7 + q] += e[q];
        }
        if (out) out[c * n_z + i] = g.val;
        const T gz1 = w * o.dz1, gz2 = w * g.dz;
        if (zstride != 0) {
            if (g1_out) g1_out[c * n_z + i] = gz1;
            if (g2_out) g2_out[c * n_z + i] = gz2;
        } else {
            gl1[k * kBlock + threadIdx.x] += gz1;
            gl2[k * kBlock + threadIdx.x] += gz2;
        }
    }
}

// Occupancy of the between-limit adjoint: the compiler's allocation (the FP32 time
// coordinate's root-chain pass takes 102 VGPRs, four waves; held to five waves it spills
// vector registers to scratch).
template <typename T, int KIND> constexpr int between_min_waves() { return 1; }

// Two passes over the (cosmology tile, z block) pairs: PASS 0 takes the cosmologies whose
// lanes all follow the root chain (between_chain_only: a loop without the quadrature
// routes, so the register allocation is that loop's), PASS 1 the others, invalid ones
// included.  For limits shared by all cosmologies, pass 0 writes the tile sums of the z1-
// and z2-gradients and pass 1 adds its own where its block had a cosmology (launched
// after pass 0 on the same stream).  Pass 0 has one block per pair; pass 1, which usually
// finds nothing to do, has up to 128 blocks per tile (grid y), which test the tile's
// records once and leave, or stride over its z blocks.
template <typename T, int KIND, int ZPT, int PASS>
__device__ __forceinline__ void between_vjp_block(int64_t b, const CosmoRec *__restrict__ recs, int64_t n_cosmo,
                                                  const T *__restrict__ z1, const T *__restrict__ z2, int64_t n_z,
                                                  int64_t zstride, const T *__restrict__ cot, T *__restrict__ pacc,
                                                  T *__restrict__ g1_out, T *__restrict__ g2_out,
                                                  T *__restrict__ g1_part, T *__restrict__ g2_part,
                                                  T *__restrict__ out, int ct, int64_t nzb, T *gl1, T *gl2) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t nwz = nzb * (kBlock / 64);
    const int64_t tile = b / nzb, zb = b - tile * nzb;
    const int64_t base = zb * (int64_t)(kBlock * ZPT) + threadIdx.x;
    const int64_t gw = zb * (kBlock / 64) + wave;
    const int64_t c0 = tile * ct;
    const int64_t c1 = c0 + ct < n_cosmo ? c0 + ct : n_cosmo;
    for (int k = 0; k < ZPT; ++k) gl1[k * kBlock + threadIdx.x] = gl2[k * kBlock + threadIdx.x] = T(0);
    bool any = false; // the same on every thread of the block
    for (int64_t c = c0; c < c1; ++c) {
        const CosmoRec &r = recs[c];
        const bool chain = r.valid && between_chain_only<T, KIND>(r);
        if (chain != (PASS == 0)) continue;
        any = true;
        T acc[kAcc];
#pragma unroll
        for (int s = 0; s < kAcc; ++s) acc[s] = T(0);
        if (PASS == 0) {
            if (r.pair) between_vjp_cosmo<T, KIND, true, ZPT, true>(r, c, z1, z2, n_z, zstride, cot, base, acc, gl1, gl2, g1_out, g2_out, out);
            else between_vjp_cosmo<T, KIND, false, ZPT, true>(r, c, z1, z2, n_z, zstride, cot, base, acc, gl1, gl2, g1_out, g2_out, out);
        } else if (r.valid) {
            if (r.pair) between_vjp_cosmo<T, KIND, true, ZPT, false>(r, c, z1, z2, n_z, zstride, cot, base, acc, gl1, gl2, g1_out, g2_out, out);
            else between_vjp_cosmo<T, KIND, false, ZPT, false>(r, c, z1, z2, n_z, zstride, cot, base, acc, gl1, gl2, g1_out, g2_out, out);
        } else {
            for (int k = 0; k < ZPT; ++k) {
                const int64_t i = base + (int64_t)k * kBlock;
                if (i >= n_z) break;
                if (out) out[c * n_z + i] = Fp<T>::nan();
                if (zstride != 0) {
                    if (g1_out) g1_out[c * n_z + i] = Fp<T>::nan();
                    if (g2_out) g2_out[c * n_z + i] = Fp<T>::nan();
                } else {
                    gl1[k * kBlock + threadIdx.x] = Fp<T>::nan();
                    gl2[k * kBlock + threadIdx.x] = Fp<T>::nan();
                }
            }
        }
        if (pacc) store_partials(acc, pacc + (c * nwz + gw) * kAcc, lane);
    }
    if (zstride == 0 && (PASS == 0 || any)) {
        for (int k = 0; k < ZPT; ++k) {
            const int64_t i = base + (int64_t)k * kBlock;
            if (i >= n_z) break;
            const T v1 = gl1[k * kBlock + threadIdx.x], v2 = gl2[k * kBlock + threadIdx.x];
            if (g1_out) {
                T *d = g1_part ? g1_part + tile * n_z + i : g1_out + i;
                *d = PASS == 0 ? v1 : *d + v1;
            }
            if (g2_out) {
                T *d = g2_part ? g2_part + tile * n_z + i : g2_out + i;
                *d = PASS == 0 ? v2 : *d + v2;
            }
        }
    }
}

template <typename T, int KIND, int ZPT, int PASS>
__global__ __launch_bounds__(kBlock, (between_min_waves<T, KIND>())) void k_between_vjp(const CosmoRec *__restrict__ recs, int64_t n_cosmo,
                                                        const T *__restrict__ z1, const T *__restrict__ z2,
                                                        int64_t n_z, int64_t zstride, const T *__restrict__ cot,
                                                        T *__restrict__ pacc, T *__restrict__ g1_out,
                                                        T *__restrict__ g2_out, T *__restrict__ g1_part,
                                                        T *__restrict__ g2_part, T *__restrict__ out, int ct,
                                                        int64_t nzb) {
    __shared__ T gl1[ZPT * kBlock], gl2[ZPT * kBlock];
    if (PASS == 0) {
        between_vjp_block<T, KIND, ZPT, 0>(blockIdx.x, recs, n_cosmo, z1, z2, n_z, zstride, cot, pacc, g1_out, g2_out,
                                           g1_part, g2_part, out, ct, nzb, gl1, gl2);
    } else {
        // grid (z-block groups, tiles): the tile's records are tested once, one per lane
        const int64_t tile = blockIdx.y;
        bool other = false;
        for (int64_t j = threadIdx.x; j < ct; j += kBlock) {
            const int64_t c = tile * ct + j;
            other |= c < n_cosmo && !(recs[c].valid && between_chain_only<T, KIND>(recs[c]));
        }
        if (!__syncthreads_or(other)) return;
        for (int64_t zb = blockIdx.x; zb < nzb; zb += gridDim.x)
            between_vjp_block<T, KIND, ZPT, 1>(tile * nzb + zb, recs, n_cosmo, z1, z2, n_z, zstride, cot, pacc,
                                               g1_out, g2_out, g1_part, g2_part, out, ct, nzb, gl1, gl2);
    }
}

// Materialised Jacobian: per lane the observable and d out / d(H0, Om0, OL0, Or0, z),
// written as five planes jac[q][c][i]; the root-space partials are contracted with the
// root Jacobian per lane (jac_contract: FP32 lanes in FP32 with a cancellation check).
// Grid as k_forward, on tiles of up to 24 cosmologies.
// Occupancy of the materialised Jacobian: the FP32 comoving-distance family held to seven
// waves (65 VGPRs, no spills; at eight, 64 VGPRs, two scalar registers spill and it ran no
// faster); the others keep the compiler's allocation.
template <typename T, int KIND> constexpr int jac_min_waves() {
    return (sizeof(T) == 4 && KIND != COSMO_T && KIND != COSMO_X) ? 7 : 1;
}

// The lane's partials contracted with the root Jacobian (app. A) per parameter, with the
// cancellation check of kJacCancel32: FP32 lanes contract in FP32 with the FP32 copies of
// the coefficients (the check compares the size of the terms with their sum, which does
// not depend on the precision of the contraction); FP64 lanes as root_contract.  Returns
// false where the terms cancel by more than kJacCancel32 (FP32 only).
template <typename T, typename D>
__device__ __forceinline__ bool jac_contract(const CosmoRec &r, const T p[5], D d[3]) {
    if (sizeof(T) == 4) {
        bool ok = true;
#pragma unroll
        for (int th = 0; th < 3; ++th) {
            // sum of the terms and of their magnitudes, one FMA each (|p c| = |p| |c|)
            float sum = 0.0f, mag = 0.0f;
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                const float c = r.jc32[q][th];
                sum = __builtin_fmaf((float)p[q], c, sum);
                mag = __builtin_fmaf(__builtin_fabsf((float)p[q]), __builtin_fabsf(c), mag);
            }
            d[th] = D(sum);
            ok = ok && (mag <= float(kJacCancel32) * __builtin_fabsf(sum));
        }
        return ok;
    }
    double pd[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) pd[q] = (double)p[q];
#pragma unroll
    for (int th = 0; th < 3; ++th) d[th] = D(root_contract(r, pd, th));
    return true;
}

template <typename T, int KIND>
__global__ __launch_bounds__(kBlock, (jac_min_waves<T, KIND>())) void k_jac(const CosmoRec *__restrict__ recs, int64_t n_cosmo,
                                                 const T *__restrict__ z, int64_t n_z, int64_t zstride,
                                                 T *__restrict__ out, T *__restrict__ jac, int32_t *__restrict__ info,
                                                 int ct, int64_t nzb) {
    // grid as k_forward
    const int64_t tile = blockIdx.y, zb = blockIdx.x;
    const int64_t i = zb * kBlock + threadIdx.x;
    const bool active = i < n_z;
    const uint32_t i32 = (uint32_t)i; // n_z < 2^29 (checked on the host)
    const int64_t c0 = tile * ct;
    const int64_t c1 = c0 + ct < n_cosmo ? c0 + ct : n_cosmo;
    const int64_t plane = n_cosmo * n_z;
    // no cross-lane work below: lanes past the end leave at once (which keeps the
    // cosmology loop uniform)
    if (!active) return;
    auto lane = [&](int64_t c, T zz) __attribute__((always_inline)) {
        const CosmoRec &r = recs[c];
        T v, J[5];
        bool used_gl = false;
        if (!r.valid) {
            v = Fp<T>::nan();
#pragma unroll
            for (int q = 0; q < 5; ++q) J[q] = Fp<T>::nan();
        } else if (KIND != COSMO_X && !adjoint_quadrature_lane<T>(KIND, r, zz)) {
            // root-chain lane (the common case)
            RootGrad<T> o;
            if (r.pair) lane_grad_root<T, KIND, true>(r, zz, o);
            else lane_grad_root<T, KIND, false>(r, zz, o);
            v = o.val;
            J[0] = o.dh;
            J[4] = o.dz;
#pragma unroll
            for (int q = 1; q < 5; ++q) o.p[q] *= o.ps;
            T d[3];
            if (!jac_contract(r, o.p, d)) {
                // the contraction cancels (small beta, small z): Leibniz-rule quadrature
                T bv, g[3];
                if (r.pair) gl_integral<T, true>(lane_of<T>(r), zz, KIND == COSMO_T ? 1 : 0, true, bv, g, 1);
                else gl_integral<T, false>(lane_of<T>(r), zz, KIND == COSMO_T ? 1 : 0, true, bv, g, 1);
#pragma unroll
                for (int th = 0; th < 3; ++th) d[th] = g[th];
            }
#pragma unroll
            for (int th = 0; th < 3; ++th) J[1 + th] = o.s * d[th] - o.dok;
        } else {
            LaneGrad<T> o;
            if (r.pair) lane_grad<T, KIND, true>(r, zz, o, used_gl);
            else lane_grad<T, KIND, false>(r, zz, o, used_gl);
            v = o.val;
            J[0] = o.dh;
            J[4] = o.dz;
            double d[3];
            if (o.quad) {
#pragma unroll
                for (int th = 0; th < 3; ++th) d[th] = o.q[th];
            } else if (!jac_contract(r, o.p, d) && KIND != COSMO_X) {
                T bv, g[3];
                if (r.pair) gl_integral<T, true>(lane_of<T>(r), zz, KIND == COSMO_T ? 1 : 0, true, bv, g, 1);
                else gl_integral<T, false>(lane_of<T>(r), zz, KIND == COSMO_T ? 1 : 0, true, bv, g, 1);
#pragma unroll
                for (int th = 0; th < 3; ++th) d[th] = g[th];
            }
#pragma unroll
            for (int th = 0; th < 3; ++th) J[1 + th] = T((double)o.s * d[th] - (double)o.dok);
        }
        T *__restrict__ row = jac + c * n_z;
        if (out) __builtin_nontemporal_store(v, (out + c * n_z) + i32);
#pragma unroll
        for (int q = 0; q < 5; ++q) __builtin_nontemporal_store(J[q], (row + q * plane) + i32);
        if (KIND == COSMO_X && info) {
            unsigned long long m = __ballot(used_gl);
            if (m && (int)__lane_id() == __ffsll((long long)m) - 1) atomicOr(info + c, COSMO_INFO_X_QUADRATURE);
        }
    };
    if (zstride == 0) {
        const T zz = z[i];
        // as in k_forward: no load, and no wait on the vector-memory counter, in the loop
        __builtin_amdgcn_s_waitcnt(0);
        for (int64_t c = c0; c < c1; ++c) lane(c, zz);
    } else {
        for (int64_t c = c0; c < c1; ++c) lane(c, (z + c * zstride)[i32]);
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_finalize_params(const CosmoRec *__restrict__ recs, int64_t n_cosmo,
                                                            const T *__restrict__ pacc, int64_t nwz,
                                                            int kind, int fp32, double *__restrict__ grad,
                                                            double *__restrict__ loglike) {
    __shared__ double red[kBlock / 64][kAcc];
    const int64_t c = blockIdx.x;
    if (c >= n_cosmo) return;
    double acc[kAcc];
#pragma unroll
    for (int s = 0; s < kAcc; ++s) acc[s] = 0.0;
    for (int64_t q = threadIdx.x; q < nwz; q += kBlock)
#pragma unroll
        for (int s = 0; s < kAcc; ++s) acc[s] += (double)pacc[(c * nwz + q) * kAcc + s];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int s = 0; s < kAcc; ++s) {
        double v = wave_sum(acc[s]);
        if (lane == 0) red[wave][s] = v;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double a[kAcc];
    for (int s = 0; s < kAcc; ++s) {
        a[s] = 0.0;
        for (int w2 = 0; w2 < kBlock / 64; ++w2) a[s] += red[w2][s];
    }
    const CosmoRec &r = recs[c];
    if (loglike) loglike[c] = r.valid ? a[kAccLoss] : __builtin_nan("");
    if (!grad) return;
    double *g = grad + 4 * c;
    if (!r.valid) {
        for (int q = 0; q < 4; ++q) g[q] = __builtin_nan("");
        return;
    }
    g[0] = a[6];
    for (int th = 0; th < 3; ++th) {
        double v;
        // root-chain lanes (none on cosmologies whose gradient is all quadrature) plus
        // the quadrature lanes
        v = (direct_mode(kind, r, fp32 != 0) ? 0.0 : root_contract(r, a, th)) + a[7 + th];
        g[1 + th] = v - a[5]; // explicit Ok in the curvature transform: dOk/dtheta = -1
    }
}

template <typename T> __global__ void k_fill_zero(T *__restrict__ p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = T(0);
}

template <typename T>
__global__ void k_reduce_gz(const T *__restrict__ part, int64_t ntile, int64_t n_z, T *__restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_z) return;
    double s = 0.0;
    for (int64_t t = 0; t < ntile; ++t) s += (double)part[t * n_z + i];
    out[i] = (T)s;
}

// ---------------------------------------------------------------- supernova model (sec. 4)
// The per-supernova part of the variational objective of the SN Ia model (fig. 4b):
// latent redshifts z = exp(zeta) drawn from the partial multivariate normal guide,
//   zeta[s][n] = a[n] + dtheta[s] . b[n] + exp(log_s[n]) eps[s][n],
// and, per draw s and supernova n, the photometric likelihood N(zhat | z, (1+z)^2 sz^2),
// the Gamma(shape, rate) redshift prior (up to its constant), the Jacobian zeta of
// z = exp(zeta) and the eps^2/2 of the guide's density.  All arithmetic in FP64; z is
// rounded once to the distance path's precision T, and the terms use that rounded z
// (the z the distance likelihood sees).
struct SniaConst {
    double sigma_z, shape, rate;
};

// One lane per supernova, the draws in a loop (the per-supernova parameters are read
// once; each draw's row of z is written coalesced).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_snia_draw(int64_t S, int64_t N, const double *__restrict__ a,
                                                      const double *__restrict__ b,
                                                      const double *__restrict__ log_s,
                                                      const double *__restrict__ dth,
                                                      const double *__restrict__ eps, T *__restrict__ z) {
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (n >= N) return;
    const double an = a[n], b0 = b[2 * n], b1 = b[2 * n + 1], sn = exp(log_s[n]);
    for (int64_t s = 0; s < S; ++s) {
        const double zeta = an + dth[2 * s] * b0 + dth[2 * s + 1] * b1 + sn * eps[s * N + n];
        z[s * N + n] = (T)exp(zeta);
    }
}

// One lane per supernova, the draws in a loop.  With G[s][n] the derivative of
//   F = sum_{s,n} term[s][n] + sum_s loglike_s(z[s])
// with respect to zeta[s][n] (grad_z[s][n] = d loglike_s / dz[s][n], from the fused
// distance likelihood, enters through dz/dzeta = z):
//   grad_a[n] = sum_s G,  grad_b[n] = sum_s G dtheta[s],  grad_log_s[n] = sum_s G s_n eps,
// and per wave the partial sums of F's terms and of sum_n G b[n] (the dtheta[s]
// gradient), part[wave][1 + 2S] (wave sums only: no block barrier).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_snia_latent(int64_t S, int64_t N, const double *__restrict__ a,
                                                        const double *__restrict__ b,
                                                        const double *__restrict__ log_s,
                                                        const double *__restrict__ dth,
                                                        const double *__restrict__ eps,
                                                        const double *__restrict__ zhat,
                                                        const T *__restrict__ gz, SniaConst k,
                                                        double *__restrict__ ga, double *__restrict__ gb,
                                                        double *__restrict__ gls, double *__restrict__ part) {
    const int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool act = n < N;
    const bool lead = (threadIdx.x & 63) == 0;
    double an = 0.0, b0 = 0.0, b1 = 0.0, sn = 0.0, zh = 0.0;
    if (act) {
        an = a[n]; b0 = b[2 * n]; b1 = b[2 * n + 1]; sn = exp(log_s[n]); zh = zhat[n];
    }
    const double isz = 1.0 / k.sigma_z;
    double vsum = 0.0, sa = 0.0, sb0 = 0.0, sb1 = 0.0, sls = 0.0;
    double *out = part + ((int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6)) * (1 + 2 * S);
    for (int64_t s = 0; s < S; ++s) {
        const double d0 = dth[2 * s], d1 = dth[2 * s + 1];
        double g = 0.0;
        if (act) {
            const double e = eps[s * N + n];
            const double zeta = an + d0 * b0 + d1 * b1 + sn * e;
            const double ez = exp(zeta);
            const double zd = (double)(T)ez;
            const double x = 1.0 + zd, ix = 1.0 / x;
            const double r = (zh - zd) * ix * isz; // (zhat - z) / ((1 + z) sigma_z)
            vsum += -0.5 * r * r - log(x * k.sigma_z) + (k.shape - 1.0) * log(zd) - k.rate * zd + zeta + 0.5 * e * e;
            // d/dz of the photometric, normalisation and prior terms
            const double dv = r * (1.0 + zh) * ix * ix * isz - ix + (k.shape - 1.0) / zd - k.rate;
            const double dl = gz ? (double)gz[s * N + n] : 0.0;
            g = (dv + dl) * ez + 1.0;
            sa += g; sb0 += g * d0; sb1 += g * d1; sls += g * sn * e;
        }
        const double p0 = wave_sum(g * b0), p1 = wave_sum(g * b1);
        if (lead) { out[1 + 2 * s] = p0; out[2 + 2 * s] = p1; }
    }
    const double v = wave_sum(vsum);
    if (lead) out[0] = v;
    if (act) {
        ga[n] = sa; gb[2 * n] = sb0; gb[2 * n + 1] = sb1; gls[n] = sls;
    }
}

__device__ __forceinline__ double block_sum(double v, double *red) {
    v = wave_sum(v);
    const int wave = threadIdx.x >> 6;
    __syncthreads(); // the previous use of red is complete
    if ((threadIdx.x & 63) == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) t += red[w];
    return t;
}

// out[q] = sum over rows of part[row][q], q < nq (one block per quantity).
__global__ __launch_bounds__(kBlock) void k_sum_parts(const double *__restrict__ part, int64_t nrow, int64_t nq,
                                                      double *__restrict__ out) {
    __shared__ double red[kBlock / 64];
    const int64_t q = blockIdx.x;
    double v = 0.0;
    for (int64_t t = threadIdx.x; t < nrow; t += kBlock) v += part[t * nq + q];
    v = block_sum(v, red);
    if (threadIdx.x == 0) out[q] = v;
}

// ---------------------------------------------------------------- Carlson entry kernels
template <typename T, int WHICH>
__global__ void k_carlson(int64_t n, const T *__restrict__ x, const T *__restrict__ y, const T *__restrict__ z,
                          const T *__restrict__ p, T *__restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    cx<T> a = mkc(x[2 * i], x[2 * i + 1]), bb = mkc(y[2 * i], y[2 * i + 1]);
    cx<T> r;
    if (WHICH == 0) r = rf_c(a, bb, mkc(z[2 * i], z[2 * i + 1]));
    else if (WHICH == 1) r = rd_c(a, bb, mkc(z[2 * i], z[2 * i + 1]));
    else if (WHICH == 2) r = rj_c(a, bb, mkc(z[2 * i], z[2 * i + 1]), mkc(p[2 * i], p[2 * i + 1]));
    else r = rc_c(a, bb);
    out[2 * i] = r.re;
    out[2 * i + 1] = r.im;
}

} // namespace cosmo

// ==================================================================== host side
using namespace cosmo;

namespace {

struct Tiling {
    int ct;
    int64_t nzb, ntile, nblocks;
};

// zpt: redshifts per lane (1 for the forward kernels; the adjoint uses 8 on long
// redshift rows).  Cosmology tiles of up to ct_max are formed while the grid keeps
// about 8192 lane-blocks of work.
Tiling tiling(int64_t n_cosmo, int64_t n_z, int zpt = 1, int ct_max = 16) {
    Tiling t;
    const int64_t span = (int64_t)kBlock * zpt;
    t.nzb = (n_z + span - 1) / span;
    if (t.nzb < 1) t.nzb = 1;
    int64_t want = (n_cosmo * t.nzb * zpt) / 8192;
    t.ct = (int)(want < 1 ? 1 : (want > ct_max ? ct_max : want));
    // at most 65535 tiles (the forward and Jacobian grids put them on the y axis)
    const int64_t ct_min = (n_cosmo + 65534) / 65535;
    if (t.ct < ct_min) t.ct = (int)ct_min;
    t.ntile = (n_cosmo + t.ct - 1) / t.ct;
    t.nblocks = t.ntile * t.nzb;
    return t;
}

int vjp_zpt(int64_t n_z) { return n_z >= 8192 ? 8 : 1; }

// Tiles of the adjoints: up to kVjpTile cosmologies (the forward and Jacobian kernels
// take up to 16).  On 256 cosmologies x 1e6 shared redshifts, tiles of 8 ran the fused
// step 3% and the gradient-only call 5% faster than tiles of 16 (twice the blocks and
// tile partials of the shared-z gradient), tiles of 24 and 32 slower.
constexpr int kVjpTile = 8;
constexpr int kBetweenVjpTile = 16;
Tiling vjp_tiling(int64_t n_cosmo, int64_t n_z) { return tiling(n_cosmo, n_z, vjp_zpt(n_z), kVjpTile); }
Tiling between_vjp_tiling(int64_t n_cosmo, int64_t n_z) {
    return tiling(n_cosmo, n_z, vjp_zpt(n_z), kBetweenVjpTile);
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct WsLayout {
    size_t recs, pacc, gzp, total;
};

WsLayout ws_layout(int64_t n_cosmo, int64_t n_z) {
    const Tiling t = vjp_tiling(n_cosmo, n_z), tb = between_vjp_tiling(n_cosmo, n_z);
    WsLayout w;
    w.recs = 0;
    w.pacc = align256(sizeof(CosmoRec) * (size_t)n_cosmo);
    w.gzp = w.pacc + align256(sizeof(double) * kAcc * (size_t)n_cosmo * (size_t)t.nzb * (kBlock / 64));
    // one tile-partial plane of the shared-z gradient (distance adjoint) or two (z1 and
    // z2, between adjoint)
    const size_t planes = (size_t)t.ntile > 2 * (size_t)tb.ntile ? (size_t)t.ntile : 2 * (size_t)tb.ntile;
    w.total = w.gzp + align256(sizeof(double) * planes * (size_t)n_z);
    return w;
}

// Device memory of cosmo_distance_vjp_noalloc, for callers that cannot allocate:
// the record table, the wave partial sums and the tile partials of a shared-z
// gradient in place of a workspace.  Every GPU the library runs on holds its own
// copy until the process ends; calls on one GPU share it (every byte a call reads is
// written by the same call first, so nothing needs clearing between calls, but calls
// that overlap in time on one GPU race).  Host code never names the array in a
// kernel argument or copy: its name is a host-side stand-in there, and the device
// address comes from hipGetSymbolAddress, resolved once per device.
constexpr size_t kScratchBytes = COSMO_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::atomic<void *> g_scratch_addr[kMaxDevices];

// Address of `scratch` on the current device (resolved on the first call there; two
// threads racing on the first call store the same address).
int scratch_address(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return COSMO_E_HIP;
    void *p = g_scratch_addr[dev].load(std::memory_order_acquire);
    if (!p) {
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return COSMO_E_HIP;
        g_scratch_addr[dev].store(p, std::memory_order_release);
    }
    *out = p;
    return COSMO_OK;
}

// Layout of the adjoint's device memory packed for the fixed scratch array: the
// partial sums in the lane precision and only the tile-partial plane this call uses.
template <typename T>
WsLayout noalloc_layout(int64_t n_cosmo, int64_t n_z, int64_t zstride, bool want_params, bool want_z) {
    Tiling t = vjp_tiling(n_cosmo, n_z);
    WsLayout w;
    w.recs = 0;
    w.pacc = align256(sizeof(CosmoRec) * (size_t)n_cosmo);
    const size_t np = want_params ? sizeof(T) * kAcc * (size_t)n_cosmo * (size_t)t.nzb * (kBlock / 64) : 0;
    w.gzp = w.pacc + align256(np);
    const bool part = want_z && zstride == 0 && t.ntile > 1 && n_z > 0;
    w.total = w.gzp + (part ? align256(sizeof(T) * (size_t)t.ntile * (size_t)n_z) : 0);
    return w;
}

bool valid_kind(int k) { return k >= COSMO_DC && k <= COSMO_VC; }
bool valid_dtype(int d) { return d == COSMO_F32 || d == COSMO_F64; }

// Scoped workspace: the caller's, or stream-ordered pool memory.
struct Workspace {
    void *ptr = nullptr;
    bool owned = false;
    hipStream_t s = nullptr;
    int acquire(void *user, size_t user_bytes, size_t need, hipStream_t stream) {
        s = stream;
        if (user) {
            if (user_bytes < need) return COSMO_E_WORKSPACE;
            ptr = user;
            return COSMO_OK;
        }
        if (hipMallocAsync(&ptr, need, stream) != hipSuccess) return COSMO_E_HIP;
        owned = true;
        return COSMO_OK;
    }
    ~Workspace() {
        if (owned && ptr) (void)hipFreeAsync(ptr, s);
    }
};

template <typename T>
int launch_forward(int kind, const CosmoRec *recs, int64_t n_cosmo, const T *z, int64_t n_z, int64_t zstride,
                   T *out, int32_t *info, hipStream_t s) {
    Tiling t = tiling(n_cosmo, n_z);
    dim3 grid((unsigned)t.nzb, (unsigned)t.ntile), block(kBlock);
#define COSMO_FWD(K) hipLaunchKernelGGL((k_forward<T, K>), grid, block, 0, s, recs, n_cosmo, z, n_z, zstride, out, info, t.ct, t.nzb)
    switch (kind) {
    case COSMO_DC: COSMO_FWD(COSMO_DC); break;
    case COSMO_DM: COSMO_FWD(COSMO_DM); break;
    case COSMO_DL: COSMO_FWD(COSMO_DL); break;
    case COSMO_MU: COSMO_FWD(COSMO_MU); break;
    case COSMO_T: COSMO_FWD(COSMO_T); break;
    case COSMO_X: COSMO_FWD(COSMO_X); break;
    case COSMO_DA: COSMO_FWD(COSMO_DA); break;
    case COSMO_VC: COSMO_FWD(COSMO_VC); break;
    }
#undef COSMO_FWD
    return hipGetLastError() == hipSuccess ? COSMO_OK : COSMO_E_HIP;
}

template <typename T>
int launch_routes(int kind, const CosmoRec *recs, int64_t n_cosmo, const T *z, int64_t n_z, int64_t zstride,
                  unsigned long long *counts, hipStream_t s) {
    const unsigned nb0 = (unsigned)((4 * n_cosmo + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_fill_zero_u64<unsigned long long>, dim3(nb0), dim3(kBlock), 0, s, counts, 4 * n_cosmo);
    if (hipGetLastError() != hipSuccess) return COSMO_E_HIP;
    if (n_z == 0) return COSMO_OK;
    Tiling t = tiling(n_cosmo, n_z);
    dim3 grid((unsigned)t.nblocks), block(kBlock);
#define COSMO_RT(K) hipLaunchKernelGGL((k_routes<T, K>), grid, block, 0, s, recs, n_cosmo, z, n_z, zstride, counts, t.ct, t.nzb)
    switch (kind) {
    case COSMO_DC: COSMO_RT(COSMO_DC); break;
    case COSMO_DM: COSMO_RT(COSMO_DM); break;
    case COSMO_DL: COSMO_RT(COSMO_DL); break;
    case COSMO_MU: COSMO_RT(COSMO_MU); break;
    case COSMO_T: COSMO_RT(COSMO_T); break;
    case COSMO_X: COSMO_RT(COSMO_X); break;
    case COSMO_DA: COSMO_RT(COSMO_DA); break;
    case COSMO_VC: COSMO_RT(COSMO_VC); break;
    }
#undef COSMO_RT
    return hipGetLastError() == hipSuccess ? COSMO_OK : COSMO_E_HIP;
}

template <typename T>
int launch_between(int kind, const CosmoRec *recs, int64_t n_cosmo, const T *z1, const T *z2, int64_t n_z,
                   int64_t zstride, T *out, hipStream_t s) {
    Tiling t = tiling(n_cosmo, n_z);
    dim3 grid((unsigned)t.nblocks), block(kBlock);
#define COSMO_BTW(K) hipLaunchKernelGGL((k_between<T, K>), grid, block, 0, s, recs, n_cosmo, z1, z2, n_z, zstride, out, t.ct, t.nzb)
    switch (kind) {
    case COSMO_DC: COSMO_BTW(COSMO_DC); break;
    case COSMO_DM: COSMO_BTW(COSMO_DM); break;
    case COSMO_DA: COSMO_BTW(COSMO_DA); break;
    case COSMO_T: COSMO_BTW(COSMO_T); break;
    }
#undef COSMO_BTW
    return hipGetLastError() == hipSuccess ? COSMO_OK : COSMO_E_HIP;
}

template <typename T>
int launch_jac(int kind, const CosmoRec *recs, int64_t n_cosmo, const T *z, int64_t n_z, int64_t zstride, T *out,
               T *jac, int32_t *info, hipStream_t s) {
    // tiles of up to 24 cosmologies (1% faster than 16 on 256 x 1e6; the forward keeps 16)
    Tiling t = tiling(n_cosmo, n_z, 1, 24);
    dim3 grid((unsigned)t.nzb, (unsigned)t.ntile), block(kBlock);
#define COSMO_JAC(K) \
    hipLaunchKernelGGL((k_jac<T, K>), grid, block, 0, s, recs, n_cosmo, z, n_z, zstride, out, jac, info, t.ct, t.nzb)
    switch (kind) {
    case COSMO_DC: COSMO_JAC(COSMO_DC); break;
    case COSMO_DM: COSMO_JAC(COSMO_DM); break;
    case COSMO_DL: COSMO_JAC(COSMO_DL); break;
    case COSMO_MU: COSMO_JAC(COSMO_MU); break;
    case COSMO_T: COSMO_JAC(COSMO_T); break;
    case COSMO_X: COSMO_JAC(COSMO_X); break;
    case COSMO_DA: COSMO_JAC(COSMO_DA); break;
    case COSMO_VC: COSMO_JAC(COSMO_VC); break;
    }
#undef COSMO_JAC
    return hipGetLastError() == hipSuccess ? COSMO_OK : COSMO_E_HIP;
}

template <typename T>
// Adjoint launch.  Likelihood mode when ivar is given: cot then holds the observed
// values (laid out as z), wc the per-cosmology weights (nullable) and loglike
// receives the per-cosmology log-likelihood.
int launch_vjp(int kind, const CosmoRec *recs, int64_t n_cosmo, const T *z, int64_t n_z, int64_t zstride,
               const T *cot, const T *ivar, const double *wc, double *loglike, T *out, double *grad_params,
               T *grad_z, int32_t *info, const WsLayout &L, char *ws, hipStream_t s) {
    const int zpt = vjp_zpt(n_z);
    Tiling t = vjp_tiling(n_cosmo, n_z);
    const bool like = ivar != nullptr;
    T *pacc = (grad_params || loglike) ? (T *)(ws + L.pacc) : nullptr;
    T *gzp = (grad_z && zstride == 0 && t.ntile > 1 && n_z > 0) ? (T *)(ws + L.gzp) : nullptr;
    dim3 grid((unsigned)t.nblocks), block(kBlock);
#define COSMO_VJP_Z(K, Z, LK)                                                                                   \
    hipLaunchKernelGGL((k_vjp<T, K, Z, LK>), grid, block, 0, s, recs, n_cosmo, z, n_z, zstride, cot, ivar, wc,  \
                       pacc, grad_z, gzp, out, info, t.ct, t.nzb)
#define COSMO_VJP(K)                                                                                            \
    if (like) {                                                                                                 \
        if (zpt == 8) COSMO_VJP_Z(K, 8, true);                                                                  \
        else COSMO_VJP_Z(K, 1, true);                                                                           \
    } else {                                                                                                    \
        if (zpt == 8) COSMO_VJP_Z(K, 8, false);                                                                 \
        else COSMO_VJP_Z(K, 1, false);                                                                          \
    }
    switch (kind) {
    case COSMO_DC: COSMO_VJP(COSMO_DC); break;
    case COSMO_DM: COSMO_VJP(COSMO_DM); break;
    case COSMO_DL: COSMO_VJP(COSMO_DL); break;
    case COSMO_MU: COSMO_VJP(COSMO_MU); break;
    case COSMO_T: COSMO_VJP(COSMO_T); break;
    case COSMO_X: COSMO_VJP(COSMO_X); break;
    case COSMO_DA: COSMO_VJP(COSMO_DA); break;
    case COSMO_VC: COSMO_VJP(COSMO_VC); break;
    }
#undef COSMO_VJP
#undef COSMO_VJP_Z
    if (hipGetLastError() != hipSuccess) return COSMO_E_HIP;
    if (pacc) {
        hipLaunchKernelGGL(k_finalize_params<T>, dim3((unsigned)n_cosmo), dim3(kBlock), 0, s, recs, n_cosmo, pacc,
                           t.nzb * (kBlock / 64), kind, (int)(sizeof(T) == 4), grad_params, loglike);
        if (hipGetLastError() != hipSuccess) return COSMO_E_HIP;
    }
    if (gzp) {
        hipLaunchKernelGGL((k_reduce_gz<T>), dim3((unsigned)((n_z + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, gzp,
                           t.ntile, n_z, grad_z);
        if (hipGetLastError() != hipSuccess) return COSMO_E_HIP;
    }
    return COSMO_OK;
}

template <typename T>
int launch_between_vjp(int kind, const CosmoRec *recs, int64_t n_cosmo, const T *z1, const T *z2, int64_t n_z,
                       int64_t zstride, const T *cot, T *out, double *grad_params, T *g1, T *g2,
                       const WsLayout &L, char *ws, hipStream_t s) {
    const int zpt = vjp_zpt(n_z);
    Tiling t = between_vjp_tiling(n_cosmo, n_z);
    T *pacc = grad_params ? (T *)(ws + L.pacc) : nullptr;
    const bool part = zstride == 0 && t.ntile > 1 && n_z > 0;
    T *p1 = (part && g1) ? (T *)(ws + L.gzp) : nullptr;
    T *p2 = (part && g2) ? (T *)(ws + L.gzp) + (size_t)t.ntile * (size_t)n_z : nullptr;
    dim3 grid((unsigned)t.nblocks), block(kBlock);
    dim3 grid1((unsigned)(t.nzb < 128 ? t.nzb : 128), (unsigned)t.ntile); // the quadrature pass
#define COSMO_BVJP_Z(K, Z)                                                                                      \
    do {                                                                                                        \
        hipLaunchKernelGGL((k_between_vjp<T, K, Z, 0>), grid, block, 0, s, recs, n_cosmo, z1, z2, n_z, zstride, \
                           cot, pacc, g1, g2, p1, p2, out, t.ct, t.nzb);                                        \
        hipLaunchKernelGGL((k_between_vjp<T, K, Z, 1>), grid1, block, 0, s, recs, n_cosmo, z1, z2, n_z,         \
                           zstride, cot, pacc, g1, g2, p1, p2, out, t.ct, t.nzb);                               \
    } while (0)
#define COSMO_BVJP(K)                                                                                           \
    if (zpt == 8) COSMO_BVJP_Z(K, 8);                                                                           \
    else COSMO_BVJP_Z(K, 1)
    switch (kind) {
    case COSMO_DC: COSMO_BVJP(COSMO_DC); break;
    case COSMO_DM: COSMO_BVJP(COSMO_DM); break;
    case COSMO_DA: COSMO_BVJP(COSMO_DA); break;
    case COSMO_T: COSMO_BVJP(COSMO_T); break;
    }
#undef COSMO_BVJP
#undef COSMO_BVJP_Z
    if (hipGetLastError() != hipSuccess) return COSMO_E_HIP;
    if (pacc) {
        hipLaunchKernelGGL(k_finalize_params<T>, dim3((unsigned)n_cosmo), dim3(kBlock), 0, s, recs, n_cosmo, pacc,
                           t.nzb * (kBlock / 64), kind, (int)(sizeof(T) == 4), grad_params, (double *)nullptr);
        if (hipGetLastError() != hipSuccess) return COSMO_E_HIP;
    }
    const dim3 rg((unsigned)((n_z + kBlock - 1) / kBlock));
    if (p1) {
        hipLaunchKernelGGL((k_reduce_gz<T>), rg, dim3(kBlock), 0, s, p1, t.ntile, n_z, g1);
        if (hipGetLastError() != hipSuccess) return COSMO_E_HIP;
    }
    if (p2) {
        hipLaunchKernelGGL((k_reduce_gz<T>), rg, dim3(kBlock), 0, s, p2, t.ntile, n_z, g2);
        if (hipGetLastError() != hipSuccess) return COSMO_E_HIP;
    }
    return COSMO_OK;
}

int launch_setup(const double *params, int64_t n_cosmo, CosmoRec *recs, int32_t *info, hipStream_t s) {
    unsigned nb = (unsigned)((n_cosmo + 63) / 64);
    hipLaunchKernelGGL(k_setup, dim3(nb), dim3(64), 0, s, params, n_cosmo, recs, info);
    return hipGetLastError() == hipSuccess ? COSMO_OK : COSMO_E_HIP;
}

template <typename T, int WHICH>
int launch_carlson(int64_t n, const void *x, const void *y, const void *z, const void *p, void *out, hipStream_t s) {
    unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL((k_carlson<T, WHICH>), dim3(nb), dim3(kBlock), 0, s, n, (const T *)x, (const T *)y,
                       (const T *)z, (const T *)p, (T *)out);
    return hipGetLastError() == hipSuccess ? COSMO_OK : COSMO_E_HIP;
}

template <int WHICH>
int carlson_entry(int dt, int64_t n, const void *x, const void *y, const void *z, const void *p, void *out,
                  void *stream) {
    if (!valid_dtype(dt)) return COSMO_E_DTYPE;
    if (n < 0 || (n > 0 && (!x || !y || !out))) return COSMO_E_ARG;
    if (n > 0 && (WHICH == 0 || WHICH == 1 || WHICH == 2) && !z) return COSMO_E_ARG;
    if (n > 0 && WHICH == 2 && !p) return COSMO_E_ARG;
    if (n == 0) return COSMO_OK;
    if (n > (int64_t)0xFFFFFFFFll * kBlock) return COSMO_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    return dt == COSMO_F32 ? launch_carlson<float, WHICH>(n, x, y, z, p, out, s)
                           : launch_carlson<double, WHICH>(n, x, y, z, p, out, s);
}

int check_grid(int64_t n_cosmo, int64_t n_z) {
    Tiling t = tiling(n_cosmo, n_z);  // the forward grid is the larger one
    if (t.nblocks > 0x7FFFFFFFll) return COSMO_E_ARG;
    if (n_cosmo > 0x7FFFFFFFll) return COSMO_E_ARG;
    if (n_z > (1ll << 29) - 8 * kBlock) return COSMO_E_ARG; // 32-bit byte offsets within a row in the kernels
    return COSMO_OK;
}

size_t snia_ws_bytes(int64_t n_draws, int64_t n_sn) {
    const int64_t nwave = (n_sn + kBlock - 1) / kBlock * (kBlock / 64);
    return align256(sizeof(double) * (size_t)nwave * (size_t)(1 + 2 * n_draws));
}

bool snia_sizes_ok(int64_t n_draws, int64_t n_sn) {
    if (n_draws < 0 || n_sn < 0) return false;
    if (n_draws > 0 && n_sn > ((int64_t)0xFFFFFFFFll * kBlock) / n_draws) return false; // (draw, SN) pairs in 32-bit block counts
    if (2 * n_draws + 1 > 0x7FFFFFFFll) return false;
    return true;
}

} // namespace

extern "C" {

const char *cosmo_version(void) { return "cosmo-carlson-gfx950 1.0"; }

int cosmo_workspace_size(int64_t n_cosmo, int64_t n_z, size_t *bytes) {
    if (!bytes || n_cosmo < 0 || n_z < 0) return COSMO_E_ARG;
    *bytes = ws_layout(n_cosmo, n_z).total;
    return COSMO_OK;
}

int cosmo_roots(const double *params, int64_t n_cosmo, double *roots, int32_t *info, void *stream) {
    if (n_cosmo < 0 || (n_cosmo > 0 && (!params || !roots))) return COSMO_E_ARG;
    if (n_cosmo == 0) return COSMO_OK;
    if (n_cosmo > 0x7FFFFFFFll) return COSMO_E_ARG;
    unsigned nb = (unsigned)((n_cosmo + 63) / 64);
    hipLaunchKernelGGL(k_roots, dim3(nb), dim3(64), 0, (hipStream_t)stream, params, n_cosmo, roots, info);
    return hipGetLastError() == hipSuccess ? COSMO_OK : COSMO_E_HIP;
}

int carlson_rf(cosmo_dtype dt, int64_t n, const void *x, const void *y, const void *z, void *out, void *stream) {
    return carlson_entry<0>(dt, n, x, y, z, nullptr, out, stream);
}
int carlson_rd(cosmo_dtype dt, int64_t n, const void *x, const void *y, const void *z, void *out, void *stream) {
    return carlson_entry<1>(dt, n, x, y, z, nullptr, out, stream);
}
int carlson_rj(cosmo_dtype dt, int64_t n, const void *x, const void *y, const void *z, const void *p, void *out,
               void *stream) {
    return carlson_entry<2>(dt, n, x, y, z, p, out, stream);
}
int carlson_rc(cosmo_dtype dt, int64_t n, const void *x, const void *y, void *out, void *stream) {
    return carlson_entry<3>(dt, n, x, y, nullptr, nullptr, out, stream);
}

int cosmo_distance(cosmo_kind kind, cosmo_dtype dt, const double *params, int64_t n_cosmo, const void *z,
                   int64_t n_z, int64_t z_cosmo_stride, void *out, int32_t *info, void *workspace,
                   size_t workspace_bytes, void *stream) {
    if (!valid_kind(kind)) return COSMO_E_KIND;
    if (!valid_dtype(dt)) return COSMO_E_DTYPE;
    if (n_cosmo < 0 || n_z < 0 || z_cosmo_stride < 0) return COSMO_E_ARG;
    if (n_cosmo > 0 && !params) return COSMO_E_ARG;
    if (n_cosmo > 0 && n_z > 0 && (!z || !out)) return COSMO_E_ARG;
    if (check_grid(n_cosmo, n_z) != COSMO_OK) return COSMO_E_ARG;
    if (n_cosmo == 0) return COSMO_OK;
    hipStream_t s = (hipStream_t)stream;
    int rc;
    WsLayout L = ws_layout(n_cosmo, 0);
    Workspace ws;
    rc = ws.acquire(workspace, workspace_bytes, L.pacc, s);
    if (rc != COSMO_OK) return rc;
    CosmoRec *recs = (CosmoRec *)ws.ptr;
    rc = launch_setup(params, n_cosmo, recs, info, s);
    if (rc != COSMO_OK || n_z == 0) return rc;
    if (dt == COSMO_F32)
        return launch_forward<float>(kind, recs, n_cosmo, (const float *)z, n_z, z_cosmo_stride, (float *)out, info, s);
    return launch_forward<double>(kind, recs, n_cosmo, (const double *)z, n_z, z_cosmo_stride, (double *)out, info, s);
}

int cosmo_route_counts(cosmo_kind kind, cosmo_dtype dt, const double *params, int64_t n_cosmo, const void *z,
                       int64_t n_z, int64_t z_cosmo_stride, int64_t *counts, void *workspace,
                       size_t workspace_bytes, void *stream) {
    if (!valid_kind(kind)) return COSMO_E_KIND;
    if (!valid_dtype(dt)) return COSMO_E_DTYPE;
    if (n_cosmo < 0 || n_z < 0 || z_cosmo_stride < 0) return COSMO_E_ARG;
    if (n_cosmo > 0 && (!params || !counts)) return COSMO_E_ARG;
    if (n_cosmo > 0 && n_z > 0 && !z) return COSMO_E_ARG;
    if (check_grid(n_cosmo, n_z) != COSMO_OK) return COSMO_E_ARG;
    if (n_cosmo == 0) return COSMO_OK;
    hipStream_t s = (hipStream_t)stream;
    WsLayout L = ws_layout(n_cosmo, n_z);
    Workspace ws;
    int rc = ws.acquire(workspace, workspace_bytes, L.pacc, s);
    if (rc != COSMO_OK) return rc;
    CosmoRec *recs = (CosmoRec *)ws.ptr;
    rc = launch_setup(params, n_cosmo, recs, nullptr, s);
    if (rc != COSMO_OK) return rc;
    unsigned long long *cnt = (unsigned long long *)counts;
    return dt == COSMO_F32 ? launch_routes<float>(kind, recs, n_cosmo, (const float *)z, n_z, z_cosmo_stride, cnt, s)
                           : launch_routes<double>(kind, recs, n_cosmo, (const double *)z, n_z, z_cosmo_stride, cnt, s);
}

int cosmo_distance_between(cosmo_kind kind, cosmo_dtype dt, const double *params, int64_t n_cosmo,
                           const void *z1, const void *z2, int64_t n_z, int64_t z_cosmo_stride, void *out,
                           int32_t *info, void *workspace, size_t workspace_bytes, void *stream) {
    if (!(kind == COSMO_DC || kind == COSMO_DM || kind == COSMO_DA || kind == COSMO_T)) return COSMO_E_KIND;
    if (!valid_dtype(dt)) return COSMO_E_DTYPE;
    if (n_cosmo < 0 || n_z < 0 || z_cosmo_stride < 0) return COSMO_E_ARG;
    if (n_cosmo > 0 && !params) return COSMO_E_ARG;
    if (n_cosmo > 0 && n_z > 0 && (!z1 || !z2 || !out)) return COSMO_E_ARG;
    if (check_grid(n_cosmo, n_z) != COSMO_OK) return COSMO_E_ARG;
    if (n_cosmo == 0) return COSMO_OK;
    hipStream_t s = (hipStream_t)stream;
    int rc;
    WsLayout L = ws_layout(n_cosmo, 0);
    Workspace ws;
    rc = ws.acquire(workspace, workspace_bytes, L.pacc, s);
    if (rc != COSMO_OK) return rc;
    CosmoRec *recs = (CosmoRec *)ws.ptr;
    rc = launch_setup(params, n_cosmo, recs, info, s);
    if (rc != COSMO_OK || n_z == 0) return rc;
    if (dt == COSMO_F32)
        return launch_between<float>(kind, recs, n_cosmo, (const float *)z1, (const float *)z2, n_z, z_cosmo_stride,
                                     (float *)out, s);
    return launch_between<double>(kind, recs, n_cosmo, (const double *)z1, (const double *)z2, n_z, z_cosmo_stride,
                                  (double *)out, s);
}

int cosmo_distance_between_vjp(cosmo_kind kind, cosmo_dtype dt, const double *params, int64_t n_cosmo,
                               const void *z1, const void *z2, int64_t n_z, int64_t z_cosmo_stride, const void *cot,
                               void *out, double *grad_params, void *grad_z1, void *grad_z2, int32_t *info,
                               void *workspace, size_t workspace_bytes, void *stream) {
    if (!(kind == COSMO_DC || kind == COSMO_DM || kind == COSMO_DA || kind == COSMO_T)) return COSMO_E_KIND;
    if (!valid_dtype(dt)) return COSMO_E_DTYPE;
    if (n_cosmo < 0 || n_z < 0 || z_cosmo_stride < 0) return COSMO_E_ARG;
    if (n_cosmo > 0 && !params) return COSMO_E_ARG;
    if (n_cosmo > 0 && n_z > 0 && (!z1 || !z2 || !cot)) return COSMO_E_ARG;
    if (check_grid(n_cosmo, n_z) != COSMO_OK) return COSMO_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (n_cosmo == 0) {
        // empty sums over cosmologies: shared-limit gradients are zero (fill kernels, no
        // memset)
        if (n_z > 0 && z_cosmo_stride == 0) {
            unsigned nb = (unsigned)((n_z + kBlock - 1) / kBlock);
            for (void *g : {grad_z1, grad_z2}) {
                if (!g) continue;
                if (dt == COSMO_F32) hipLaunchKernelGGL(k_fill_zero<float>, dim3(nb), dim3(kBlock), 0, s, (float *)g, n_z);
                else hipLaunchKernelGGL(k_fill_zero<double>, dim3(nb), dim3(kBlock), 0, s, (double *)g, n_z);
            }
        }
        return hipGetLastError() == hipSuccess ? COSMO_OK : COSMO_E_HIP;
    }
    int rc;
    WsLayout L = ws_layout(n_cosmo, n_z);
    Workspace ws;
    rc = ws.acquire(workspace, workspace_bytes, L.total, s);
    if (rc != COSMO_OK) return rc;
    CosmoRec *recs = (CosmoRec *)ws.ptr;
    rc = launch_setup(params, n_cosmo, recs, info, s);
    if (rc != COSMO_OK) return rc;
    if (dt == COSMO_F32)
        return launch_between_vjp<float>(kind, recs, n_cosmo, (const float *)z1, (const float *)z2, n_z,
                                         z_cosmo_stride, (const float *)cot, (float *)out, grad_params,
                                         (float *)grad_z1, (float *)grad_z2, L, (char *)ws.ptr, s);
    return launch_between_vjp<double>(kind, recs, n_cosmo, (const double *)z1, (const double *)z2, n_z,
                                      z_cosmo_stride, (const double *)cot, (double *)out, grad_params,
                                      (double *)grad_z1, (double *)grad_z2, L, (char *)ws.ptr, s);
}

int cosmo_distance_vjp(cosmo_kind kind, cosmo_dtype dt, const double *params, int64_t n_cosmo, const void *z,
                       int64_t n_z, int64_t z_cosmo_stride, const void *cot, void *out, double *grad_params,
                       void *grad_z, int32_t *info, void *workspace, size_t workspace_bytes, void *stream) {
    if (!valid_kind(kind)) return COSMO_E_KIND;
    if (!valid_dtype(dt)) return COSMO_E_DTYPE;
    if (n_cosmo < 0 || n_z < 0 || z_cosmo_stride < 0) return COSMO_E_ARG;
    if (n_cosmo > 0 && !params) return COSMO_E_ARG;
    if (n_cosmo > 0 && n_z > 0 && (!z || !cot)) return COSMO_E_ARG;
    if (check_grid(n_cosmo, n_z) != COSMO_OK) return COSMO_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (n_cosmo == 0) {
        // empty sum over cosmologies: a shared-z gradient is zero (fill kernel, no memset,
        // so that the call stays capturable in a HIP graph)
        if (grad_z && n_z > 0 && z_cosmo_stride == 0) {
            unsigned nb = (unsigned)((n_z + kBlock - 1) / kBlock);
            if (dt == COSMO_F32) hipLaunchKernelGGL(k_fill_zero<float>, dim3(nb), dim3(kBlock), 0, s, (float *)grad_z, n_z);
            else hipLaunchKernelGGL(k_fill_zero<double>, dim3(nb), dim3(kBlock), 0, s, (double *)grad_z, n_z);
            if (hipGetLastError() != hipSuccess) return COSMO_E_HIP;
        }
        return COSMO_OK;
    }
    int rc;
    WsLayout L = ws_layout(n_cosmo, n_z);
    Workspace ws;
    rc = ws.acquire(workspace, workspace_bytes, L.total, s);
    if (rc != COSMO_OK) return rc;
    CosmoRec *recs = (CosmoRec *)ws.ptr;
    rc = launch_setup(params, n_cosmo, recs, info, s);
    if (rc != COSMO_OK) return rc;
    if (dt == COSMO_F32)
        return launch_vjp<float>(kind, recs, n_cosmo, (const float *)z, n_z, z_cosmo_stride, (const float *)cot,
                                 nullptr, nullptr, nullptr, (float *)out, grad_params, (float *)grad_z, info, L,
                                 (char *)ws.ptr, s);
    return launch_vjp<double>(kind, recs, n_cosmo, (const double *)z, n_z, z_cosmo_stride, (const double *)cot,
                              nullptr, nullptr, nullptr, (double *)out, grad_params, (double *)grad_z, info, L,
                              (char *)ws.ptr, s);
}

int cosmo_distance_vjp_noalloc(cosmo_kind kind, cosmo_dtype dt, const double *params, int64_t n_cosmo,
                               const void *z, int64_t n_z, int64_t z_cosmo_stride, const void *cot, void *out,
                               double *grad_params, void *grad_z, int32_t *info, void *stream) {
    if (!valid_kind(kind)) return COSMO_E_KIND;
    if (!valid_dtype(dt)) return COSMO_E_DTYPE;
    if (n_cosmo < 0 || n_z < 0 || z_cosmo_stride < 0) return COSMO_E_ARG;
    if (n_cosmo > 0 && !params) return COSMO_E_ARG;
    if (n_cosmo > 0 && n_z > 0 && (!z || !cot)) return COSMO_E_ARG;
    if (check_grid(n_cosmo, n_z) != COSMO_OK) return COSMO_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (n_cosmo == 0) {
        if (grad_z && n_z > 0 && z_cosmo_stride == 0) {
            unsigned nb = (unsigned)((n_z + kBlock - 1) / kBlock);
            if (dt == COSMO_F32) hipLaunchKernelGGL(k_fill_zero<float>, dim3(nb), dim3(kBlock), 0, s, (float *)grad_z, n_z);
            else hipLaunchKernelGGL(k_fill_zero<double>, dim3(nb), dim3(kBlock), 0, s, (double *)grad_z, n_z);
            if (hipGetLastError() != hipSuccess) return COSMO_E_HIP;
        }
        return COSMO_OK;
    }
    const WsLayout L = dt == COSMO_F32
                           ? noalloc_layout<float>(n_cosmo, n_z, z_cosmo_stride, grad_params != nullptr, grad_z != nullptr)
                           : noalloc_layout<double>(n_cosmo, n_z, z_cosmo_stride, grad_params != nullptr, grad_z != nullptr);
    // checked before any HIP call: a problem beyond the fixed array is refused whole
    if (L.total > kScratchBytes) return COSMO_E_SCRATCH;
    void *base = nullptr;
    int rc = scratch_address(&base);
    if (rc != COSMO_OK) return rc;
    CosmoRec *recs = (CosmoRec *)base;
    rc = launch_setup(params, n_cosmo, recs, info, s);
    if (rc != COSMO_OK) return rc;
    if (dt == COSMO_F32)
        return launch_vjp<float>(kind, recs, n_cosmo, (const float *)z, n_z, z_cosmo_stride, (const float *)cot,
                                 nullptr, nullptr, nullptr, (float *)out, grad_params, (float *)grad_z, info, L,
                                 (char *)base, s);
    return launch_vjp<double>(kind, recs, n_cosmo, (const double *)z, n_z, z_cosmo_stride, (const double *)cot,
                              nullptr, nullptr, nullptr, (double *)out, grad_params, (double *)grad_z, info, L,
                              (char *)base, s);
}

int cosmo_distance_jac(cosmo_kind kind, cosmo_dtype dt, const double *params, int64_t n_cosmo, const void *z,
                       int64_t n_z, int64_t z_cosmo_stride, void *out, void *jac, int32_t *info, void *workspace,
                       size_t workspace_bytes, void *stream) {
    if (!valid_kind(kind)) return COSMO_E_KIND;
    if (!valid_dtype(dt)) return COSMO_E_DTYPE;
    if (n_cosmo < 0 || n_z < 0 || z_cosmo_stride < 0) return COSMO_E_ARG;
    if (n_cosmo > 0 && !params) return COSMO_E_ARG;
    if (n_cosmo > 0 && n_z > 0 && (!z || !jac)) return COSMO_E_ARG;
    if (check_grid(n_cosmo, n_z) != COSMO_OK) return COSMO_E_ARG;
    if (n_cosmo == 0) return COSMO_OK;
    hipStream_t s = (hipStream_t)stream;
    int rc;
    WsLayout L = ws_layout(n_cosmo, 0);
    Workspace ws;
    rc = ws.acquire(workspace, workspace_bytes, L.pacc, s);
    if (rc != COSMO_OK) return rc;
    CosmoRec *recs = (CosmoRec *)ws.ptr;
    rc = launch_setup(params, n_cosmo, recs, info, s);
    if (rc != COSMO_OK || n_z == 0) return rc;
    if (dt == COSMO_F32)
        return launch_jac<float>(kind, recs, n_cosmo, (const float *)z, n_z, z_cosmo_stride, (float *)out,
                                 (float *)jac, info, s);
    return launch_jac<double>(kind, recs, n_cosmo, (const double *)z, n_z, z_cosmo_stride, (double *)out,
                              (double *)jac, info, s);
}

int cosmo_gaussian_loglike(cosmo_kind kind, cosmo_dtype dt, const double *params, int64_t n_cosmo, const void *z,
                           int64_t n_z, int64_t z_cosmo_stride, const void *obs, const void *ivar, const double *wc,
                           double *loglike, double *grad_params, void *grad_z, int32_t *info, void *workspace,
                           size_t workspace_bytes, void *stream) {
    if (!valid_kind(kind)) return COSMO_E_KIND;
    if (!valid_dtype(dt)) return COSMO_E_DTYPE;
    if (n_cosmo < 0 || n_z < 0 || z_cosmo_stride < 0) return COSMO_E_ARG;
    if (n_cosmo > 0 && !params) return COSMO_E_ARG;
    if (n_cosmo > 0 && n_z > 0 && (!z || !obs || !ivar)) return COSMO_E_ARG;
    if (check_grid(n_cosmo, n_z) != COSMO_OK) return COSMO_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (n_cosmo == 0 || n_z == 0) {
        // empty sums: zero log-likelihoods and gradients (fill kernels, no memset)
        if (n_cosmo > 0) {
            unsigned nb = (unsigned)((4 * n_cosmo + kBlock - 1) / kBlock);
            if (loglike) hipLaunchKernelGGL(k_fill_zero<double>, dim3(nb), dim3(kBlock), 0, s, loglike, n_cosmo);
            if (grad_params) hipLaunchKernelGGL(k_fill_zero<double>, dim3(nb), dim3(kBlock), 0, s, grad_params, 4 * n_cosmo);
        }
        if (grad_z && n_z > 0 && z_cosmo_stride == 0) {
            unsigned nb = (unsigned)((n_z + kBlock - 1) / kBlock);
            if (dt == COSMO_F32) hipLaunchKernelGGL(k_fill_zero<float>, dim3(nb), dim3(kBlock), 0, s, (float *)grad_z, n_z);
            else hipLaunchKernelGGL(k_fill_zero<double>, dim3(nb), dim3(kBlock), 0, s, (double *)grad_z, n_z);
        }
        return hipGetLastError() == hipSuccess ? COSMO_OK : COSMO_E_HIP;
    }
    int rc;
    WsLayout L = ws_layout(n_cosmo, n_z);
    Workspace ws;
    rc = ws.acquire(workspace, workspace_bytes, L.total, s);
    if (rc != COSMO_OK) return rc;
    CosmoRec *recs = (CosmoRec *)ws.ptr;
    rc = launch_setup(params, n_cosmo, recs, info, s);
    if (rc != COSMO_OK) return rc;
    if (dt == COSMO_F32)
        return launch_vjp<float>(kind, recs, n_cosmo, (const float *)z, n_z, z_cosmo_stride, (const float *)obs,
                                 (const float *)ivar, wc, loglike, nullptr, grad_params, (float *)grad_z, info, L,
                                 (char *)ws.ptr, s);
    return launch_vjp<double>(kind, recs, n_cosmo, (const double *)z, n_z, z_cosmo_stride, (const double *)obs,
                              (const double *)ivar, wc, loglike, nullptr, grad_params, (double *)grad_z, info, L,
                              (char *)ws.ptr, s);
}


int snia_workspace_size(int64_t n_draws, int64_t n_sn, size_t *bytes) {
    if (!bytes || !snia_sizes_ok(n_draws, n_sn)) return COSMO_E_ARG;
    *bytes = snia_ws_bytes(n_draws, n_sn);
    return COSMO_OK;
}

int snia_draw(cosmo_dtype dt, int64_t n_draws, int64_t n_sn, const double *a, const double *b, const double *log_s,
              const double *dtheta, const double *eps, void *z, void *stream) {
    if (!valid_dtype(dt)) return COSMO_E_DTYPE;
    if (!snia_sizes_ok(n_draws, n_sn)) return COSMO_E_ARG;
    if (n_draws == 0 || n_sn == 0) return COSMO_OK;
    if (!a || !b || !log_s || !dtheta || !eps || !z) return COSMO_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    const dim3 grid((unsigned)((n_sn + kBlock - 1) / kBlock));
    if (dt == COSMO_F32) hipLaunchKernelGGL(k_snia_draw<float>, grid, dim3(kBlock), 0, s, n_draws, n_sn, a, b, log_s, dtheta, eps, (float *)z);
    else hipLaunchKernelGGL(k_snia_draw<double>, grid, dim3(kBlock), 0, s, n_draws, n_sn, a, b, log_s, dtheta, eps, (double *)z);
    return hipGetLastError() == hipSuccess ? COSMO_OK : COSMO_E_HIP;
}

int snia_latent_vjp(cosmo_dtype dt, int64_t n_draws, int64_t n_sn, const double *a, const double *b,
                    const double *log_s, const double *dtheta, const double *eps, const double *zhat,
                    const void *grad_z, double sigma_z, double gamma_shape, double gamma_rate,
                    double *value_dtheta, double *grad_a, double *grad_b, double *grad_log_s, void *workspace,
                    size_t workspace_bytes, void *stream) {
    if (!valid_dtype(dt)) return COSMO_E_DTYPE;
    if (!snia_sizes_ok(n_draws, n_sn)) return COSMO_E_ARG;
    if (!(sigma_z > 0.0) || !(gamma_shape > 0.0) || !(gamma_rate > 0.0) || !__builtin_isfinite(sigma_z) ||
        !__builtin_isfinite(gamma_shape) || !__builtin_isfinite(gamma_rate))
        return COSMO_E_ARG;
    if (!value_dtheta) return COSMO_E_ARG;
    if (n_sn > 0 && (!grad_a || !grad_b || !grad_log_s)) return COSMO_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (n_draws == 0 || n_sn == 0) {
        // empty sums (fill kernels, no memset)
        const int64_t nq = 1 + 2 * n_draws;
        hipLaunchKernelGGL(k_fill_zero<double>, dim3((unsigned)((nq + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                           value_dtheta, nq);
        if (n_sn > 0) {
            const dim3 g1((unsigned)((n_sn + kBlock - 1) / kBlock)), g2((unsigned)((2 * n_sn + kBlock - 1) / kBlock));
            hipLaunchKernelGGL(k_fill_zero<double>, g1, dim3(kBlock), 0, s, grad_a, n_sn);
            hipLaunchKernelGGL(k_fill_zero<double>, g2, dim3(kBlock), 0, s, grad_b, 2 * n_sn);
            hipLaunchKernelGGL(k_fill_zero<double>, g1, dim3(kBlock), 0, s, grad_log_s, n_sn);
        }
        return hipGetLastError() == hipSuccess ? COSMO_OK : COSMO_E_HIP;
    }
    if (!a || !b || !log_s || !dtheta || !eps || !zhat) return COSMO_E_ARG;
    Workspace ws;
    int rc = ws.acquire(workspace, workspace_bytes, snia_ws_bytes(n_draws, n_sn), s);
    if (rc != COSMO_OK) return rc;
    double *part = (double *)ws.ptr;
    const int64_t nblk = (n_sn + kBlock - 1) / kBlock;
    const SniaConst k{sigma_z, gamma_shape, gamma_rate};
    if (dt == COSMO_F32)
        hipLaunchKernelGGL(k_snia_latent<float>, dim3((unsigned)nblk), dim3(kBlock), 0, s, n_draws, n_sn, a, b, log_s,
                           dtheta, eps, zhat, (const float *)grad_z, k, grad_a, grad_b, grad_log_s, part);
    else
        hipLaunchKernelGGL(k_snia_latent<double>, dim3((unsigned)nblk), dim3(kBlock), 0, s, n_draws, n_sn, a, b,
                           log_s, dtheta, eps, zhat, (const double *)grad_z, k, grad_a, grad_b, grad_log_s, part);
    if (hipGetLastError() != hipSuccess) return COSMO_E_HIP;
    hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)(1 + 2 * n_draws)), dim3(kBlock), 0, s, part,
                       nblk * (kBlock / 64), 1 + 2 * n_draws, value_dtheta);
    return hipGetLastError() == hipSuccess ? COSMO_OK : COSMO_E_HIP;
}

} // extern "C"
