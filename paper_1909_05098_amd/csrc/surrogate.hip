// Learned surrogate for gfx950: a 3-level 3-D convolutional encoder-decoder
// trained and run by hand-written kernels.  Convolutions are implicit GEMMs
// on the matrix cores (v_mfma_f32_16x16x32_bf16: BF16 operands, FP32
// accumulation):
//   forward   M = voxels, N = output channels, K = 27 * input channels
//             (offset-major, channel-minor), each lane loading 8 consecutive
//             input channels of one voxel (16 bytes, channels-last); on
//             grids of 16k a persistent brick kernel (k_conv_p, k_conv_p8)
//             with the halo and a chunk's weights in LDS, which also writes
//             the pooled means of its output and reads upsampled input
//             channels at their parent voxel; gathered kernels otherwise;
//   data grad the same kernels with the weights flipped in space and
//             transposed in channels (a 3x3x3 correlation of the gradient);
//   weight grad M = output channels, N = 27 * input channels + 1 (the
//             bias), K = voxels: bricks (or 128-voxel chunks) of the
//             gradient and of the input are transposed in registers and
//             staged in LDS so that each lane reads 8 consecutive voxels of
//             one channel; partial sums per voxel split are reduced in a
//             fixed order (bit-reproducible).
// The remaining kernels are memory-bound elementwise passes: ReLU backward,
// pooling, upsampling (on small grids), the 1x1x1 head, the masked loss,
// Adam, weight packing, input rasterisation and the resampling of FED-FEM
// fields.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/fedfem.h"
#include "../../include/fedfem_surrogate.h"
#include "handle.h"
#include "internal.h"

namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16x8 zero8() {
    bf16x8 v;
#pragma unroll
    for (int j = 0; j < 8; j++) v[j] = (bf16)0.0f;
    return v;
}

inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }
inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// ---------------------------------------------------------------------------
// Convolution forward / data gradient
// ---------------------------------------------------------------------------
struct ConvArgs {
    const bf16* in;
    int ip, io, cin;  // input pitch, channel offset, channels (multiple of 8)
    const bf16* w;    // [cout][kp], k = offset * cin + ci, zero beyond 27 cin
    int kp;
    // the same weights in the brick kernel's order (k_pack_w), or null
    const uint4* wp;
    // input channels [0, upc) taken from `up` at half resolution (a 2 x 2 x 2
    // upsampling read in place: voxel v reads its parent), pitch upp, offset
    // upo; upc = 0: none (only the brick kernels take upc > 0)
    const bf16* up = nullptr;
    int upp = 0, upo = 0, upc = 0;
    // also the 2 x 2 x 2 mean of the output, [V / 8][pp] (only the brick
    // kernel), or null
    bf16* pool = nullptr;
    int pp = 0;
    // output element kept only where mk (a ReLU's output, pitch mkp, offset
    // mko) is positive: the backward of that ReLU applied to the stored BF16
    // value (only the brick kernel), or null
    const bf16* mk = nullptr;
    int mkp = 0, mko = 0;
    const float* bias;  // may be null
    bf16* out;
    int op, oo, cout;   // output pitch, channel offset, channels
    int G, ks, relu;    // grid edge, kernel size (1 or 3), ReLU on output
    int64_t V;          // voxels (batch * G^3)
};

// Each wave computes 64 voxels x (16 NT) channels; a workgroup of 4 waves
// covers 256 voxels; blockIdx.y selects a block of 64 output channels.
template <int NT>
__global__ void __launch_bounds__(256) k_conv_fwd(ConvArgs a) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t vb = ((int64_t)blockIdx.x * 4 + wave) * 64;
    const int n0 = blockIdx.y * 64;
    const int G = a.G;
    const int64_t G3 = (int64_t)G * G * G;
    int64_t vbat[4];
    int vz[4], vy[4], vx[4];
    bool ok[4];
#pragma unroll
    for (int mt = 0; mt < 4; mt++) {
        const int64_t v = vb + mt * 16 + (lane & 15);
        ok[mt] = v < a.V;
        const int64_t vv = ok[mt] ? v : 0;
        vbat[mt] = vv / G3;
        const int64_t r = vv - vbat[mt] * G3;
        vz[mt] = (int)(r / ((int64_t)G * G));
        vy[mt] = (int)((r / G) % G);
        vx[mt] = (int)(r % G);
    }
    f32x4 acc[4][NT];
#pragma unroll
    for (int mt = 0; mt < 4; mt++)
#pragma unroll
        for (int nt = 0; nt < NT; nt++) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int kg = (lane >> 4) * 8;
    const int K = (a.ks == 3 ? 27 : 1) * a.cin;
    // operands of K-step kc: the gathered input (A) and the weights (B)
    auto load = [&](int kc, bf16x8 (&A)[4], bf16x8 (&B)[NT]) {
        const int k = kc + kg;
        if (k < K) {
            const int off = k / a.cin;
            const int ci = k - off * a.cin;
            int dz = 0, dy = 0, dx = 0;
            if (a.ks == 3) {
                dz = off / 9 - 1;
                dy = (off / 3) % 3 - 1;
                dx = off % 3 - 1;
            }
#pragma unroll
            for (int mt = 0; mt < 4; mt++) {
                const int z2 = vz[mt] + dz, y2 = vy[mt] + dy, x2 = vx[mt] + dx;
                const bool in = ok[mt] && z2 >= 0 && z2 < G && y2 >= 0 && y2 < G && x2 >= 0 &&
                                x2 < G;
                if (in) {
                    const int64_t nv = ((vbat[mt] * G + z2) * G + y2) * G + x2;
                    A[mt] = *reinterpret_cast<const bf16x8*>(a.in + nv * a.ip + a.io + ci);
                } else {
                    A[mt] = zero8();
                }
            }
        } else {
#pragma unroll
            for (int mt = 0; mt < 4; mt++) A[mt] = zero8();
        }
#pragma unroll
        for (int nt = 0; nt < NT; nt++) {
            // a column past cout reads row cout - 1 instead: it only feeds
            // output channels that are never stored, and an unconditional
            // load keeps the prefetch distance (a masked one must be waited
            // for where it is masked)
            const int co = min(n0 + nt * 16 + (lane & 15), a.cout - 1);
            B[nt] = *reinterpret_cast<const bf16x8*>(a.w + (int64_t)co * a.kp + k);
        }
    };
    bf16x8 A[4], B[NT];
    load(0, A, B);
    for (int kc = 0; kc < a.kp; kc += 32) {
        // the next K-step's loads are in flight while this one multiplies
        bf16x8 An[4], Bn[NT];
        if (kc + 32 < a.kp) load(kc + 32, An, Bn);
#pragma unroll
        for (int mt = 0; mt < 4; mt++)
#pragma unroll
            for (int nt = 0; nt < NT; nt++)
                acc[mt][nt] =
                    __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mt], B[nt], acc[mt][nt], 0, 0, 0);
        if (kc + 32 < a.kp) {
#pragma unroll
            for (int mt = 0; mt < 4; mt++) A[mt] = An[mt];
#pragma unroll
            for (int nt = 0; nt < NT; nt++) B[nt] = Bn[nt];
        }
    }
    // C layout: lane holds rows (lane / 16) * 4 + i, column lane % 16
#pragma unroll
    for (int mt = 0; mt < 4; mt++)
#pragma unroll
        for (int nt = 0; nt < NT; nt++) {
            const int co = n0 + nt * 16 + (lane & 15);
            if (co >= a.cout) continue;
            const float bias = a.bias ? a.bias[co] : 0.0f;
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int64_t v = vb + mt * 16 + (lane >> 4) * 4 + i;
                if (v >= a.V) continue;
                float val = acc[mt][nt][i] + bias;
                if (a.relu) val = fmaxf(val, 0.0f);
                a.out[v * a.op + a.oo + co] = (bf16)val;
            }
        }
}

// LDS-staged 3x3x3 convolution for cin % 32 == 0 and G >= 8.  A workgroup
// owns a brick of 256 voxels of one sample (BX x BY x BZ, x fastest) and
// walks the input channels 32 at a time: it stages the brick and its one-
// voxel halo in LDS as four planes of 16-byte channel groups (plane g holds
// channels 8g..8g+7 of every halo voxel, so the 16 consecutive voxels of a
// fragment read 256 contiguous bytes and the offset enters the address
// linearly), then for each of the 27 offsets every wave reads its four
// 16-voxel A fragments from LDS (K = the 32 channels of that offset) and the
// weights from global memory (shared by all waves, so mostly cache hits).
// Each wave computes 64 voxels x (16 NT) output channels; blockIdx.y selects
// 64 output channels.
constexpr int kHaloMax = 720;  // (2+2) x (8+2) x (16+2)

template <int NT>
__global__ void __launch_bounds__(256) k_conv_lds(ConvArgs a, int BX, int BY, int BZ) {
    __shared__ bf16x8 halo[4][kHaloMax];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int G = a.G;
    const int HX = BX + 2, HY = BY + 2, HZ = BZ + 2, H = HX * HY * HZ;
    const int nbx = G / BX, nby = G / BY, nbz = G / BZ;
    int64_t id = blockIdx.x;
    const int bx = (int)(id % nbx), by = (int)((id / nbx) % nby),
              bz = (int)((id / ((int64_t)nbx * nby)) % nbz);
    const int64_t bs = id / ((int64_t)nbx * nby * nbz);
    const int x0 = bx * BX, y0 = by * BY, z0 = bz * BZ;
    const int n0 = blockIdx.y * 64;
    // this lane's four voxels (rows lane % 16 of the wave's four M tiles)
    int hv[4];
#pragma unroll
    for (int mt = 0; mt < 4; mt++) {
        const int li = wave * 64 + mt * 16 + (lane & 15);
        const int lx = li % BX, ly = (li / BX) % BY, lz = li / (BX * BY);
        hv[mt] = ((lz + 1) * HY + (ly + 1)) * HX + (lx + 1);  // halo index of offset 0
    }
    f32x4 acc[4][NT];
#pragma unroll
    for (int mt = 0; mt < 4; mt++)
#pragma unroll
        for (int nt = 0; nt < NT; nt++) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int kg = (lane >> 4) * 8;
    // weight fragments of offset `off` come from memory (L2) and are fetched
    // two offsets ahead through a ring of three register sets; the halo
    // fragments come from LDS one offset ahead
    auto loadB = [&](int c0, int off, bf16x8 (&B)[NT]) {
        const int k = off * a.cin + c0 + kg;
#pragma unroll
        for (int nt = 0; nt < NT; nt++) {
            // a column past cout reads row cout - 1 instead: it only feeds
            // output channels that are never stored, and an unconditional
            // load keeps the prefetch distance (a masked one must be waited
            // for where it is masked)
            const int co = min(n0 + nt * 16 + (lane & 15), a.cout - 1);
            B[nt] = *reinterpret_cast<const bf16x8*>(a.w + (int64_t)co * a.kp + k);
        }
    };
    auto loadA = [&](int off, bf16x8 (&A)[4]) {
        const int dz = off / 9 - 1, dy = (off / 3) % 3 - 1, dx = off % 3 - 1;
        const int dh = (dz * HY + dy) * HX + dx;
#pragma unroll
        for (int mt = 0; mt < 4; mt++)
            A[mt] = halo[lane >> 4][hv[mt] + dh];
    };
    bf16x8 Bq[3][NT];
    for (int c0 = 0; c0 < a.cin; c0 += 32) {
        loadB(c0, 0, Bq[0]);
        loadB(c0, 1, Bq[1]);
        __syncthreads();  // the previous chunk's fragments have been read
        // 64 consecutive threads stage 16 consecutive halo voxels x 4 groups
#pragma unroll 4
        for (int q = t; q < ((H + 15) >> 4) * 64; q += 256) {
            // branch-free, so several loads are in flight: lanes past the
            // halo redo its last voxel (same value, same place), and lanes
            // outside the grid load a clamped voxel and store zeros
            const int h = min((q >> 6) * 16 + (q & 15), H - 1), grp = (q >> 4) & 3;
            const int hx = h % HX, hy = (h / HX) % HY, hz = h / (HX * HY);
            const int x = x0 + hx - 1, y = y0 + hy - 1, z = z0 + hz - 1;
            const unsigned keep =
                (x >= 0 && x < G && y >= 0 && y < G && z >= 0 && z < G) ? ~0u : 0u;
            const int xc = min(max(x, 0), G - 1), yc = min(max(y, 0), G - 1),
                      zc = min(max(z, 0), G - 1);
            const int64_t gv = ((bs * G + zc) * G + yc) * G + xc;
            uint4 v = *reinterpret_cast<const uint4*>(a.in + gv * a.ip + a.io + c0 + grp * 8);
            v.x &= keep;
            v.y &= keep;
            v.z &= keep;
            v.w &= keep;
            *reinterpret_cast<uint4*>(&halo[grp][h]) = v;
        }
        __syncthreads();
        bf16x8 A[4];
        loadA(0, A);
#pragma unroll
        for (int off = 0; off < 27; off++) {
            if (off + 2 < 27) loadB(c0, off + 2, Bq[(off + 2) % 3]);
            bf16x8 An[4];
            if (off + 1 < 27) loadA(off + 1, An);
            // the prefetches stay here; the scheduler would otherwise move
            // them next to their first use
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int mt = 0; mt < 4; mt++)
#pragma unroll
                for (int nt = 0; nt < NT; nt++)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mt], Bq[off % 3][nt],
                                                                          acc[mt][nt], 0, 0, 0);
            if (off + 1 < 27) {
#pragma unroll
                for (int mt = 0; mt < 4; mt++) A[mt] = An[mt];
            }
        }
    }
    // C layout: lane holds rows (lane / 16) * 4 + i, column lane % 16
#pragma unroll
    for (int mt = 0; mt < 4; mt++)
#pragma unroll
        for (int nt = 0; nt < NT; nt++) {
            const int co = n0 + nt * 16 + (lane & 15);
            if (co >= a.cout) continue;
            const float bias = a.bias ? a.bias[co] : 0.0f;
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int li = wave * 64 + mt * 16 + (lane >> 4) * 4 + i;
                const int lx = li % BX, ly = (li / BX) % BY, lz = li / (BX * BY);
                const int64_t v = ((bs * G + z0 + lz) * G + y0 + ly) * G + x0 + lx;
                float val = acc[mt][nt][i] + bias;
                if (a.relu) val = fmaxf(val, 0.0f);
                a.out[v * a.op + a.oo + co] = (bf16)val;
            }
        }
}

// LDS-staged convolution with a chunk's whole weight set in LDS, persistent.
// A workgroup of 8 waves owns, in turn, a run of units: a brick of
// 16 x 4 x 8 voxels (wave w: z plane w, its four 16-voxel rows the M tiles)
// times a block of 32 output channels.  For each chunk of 32 input channels
// the brick's halo (18 x 6 x 10 voxels as four planes of 16-byte channel
// groups, 69 KB) and the chunk's weights for all 27 offsets (as planes of
// 8-channel groups so that 16 lanes read 256 contiguous bytes, 55 KB) sit in
// LDS; the waves run the 27 offsets without a barrier while the next item's
// halo and, when the chunk or the output block changes, its weights are in
// flight into registers, stored to LDS between two barriers at the item's
// end.  A unit's outputs leave through a 4 KB LDS slot per wave, as 16-byte
// rows of eight outputs, and, for a layer whose output is pooled, their
// 2 x 2 x 2 means too (read from the slots at the next item's end barrier).  Within a dz plane the offsets go in three dx groups: output row mt
// at dy reads halo row mt + dy, so a group reads six halo rows once for all
// three dy.  156 KB of LDS and two waves per SIMD: one workgroup per CU, 32
// per XCD.  Workgroups are dealt to the 8 XCDs round-robin; XCD x owns the
// bricks [x nb / 8, (x + 1) nb / 8) (x fastest) and its units in output-
// block-major order, each workgroup a contiguous run of them, so a run
// changes weights rarely and neighbouring bricks' halos meet in the XCD's
// L2.  Each voxel's sum goes chunk by chunk, offsets in a fixed order, so
// the result does not depend on the batch or the grid of workgroups.
constexpr int kPBX = 16, kPBY = 4, kPBZ = 8;
constexpr int kPHX = kPBX + 2, kPHY = kPBY + 2, kPHZ = kPBZ + 2;
constexpr int kPH = kPHX * kPHY * kPHZ;        // 1080 halo voxels
constexpr int kPHalo = (kPH + 15) / 16 * 64;   // staged 16-byte loads
constexpr int kPSPT = (kPHalo + 511) / 512;    // per thread: 9
constexpr int kPWts = 27 * 4 * 32;             // a chunk's weights, 16-byte elements
constexpr int kPWPT = (kPWts + 511) / 512;     // per thread: 7
constexpr int kPWGPerXcd = 32;

__global__ void __launch_bounds__(512) k_conv_p(ConvArgs a, int per) {
    __shared__ bf16x8 halo[4][kPH];
    __shared__ bf16x8 wl[27][4][32];
    __shared__ __align__(16) bf16 ep[8][64 * 32];  // per wave: its 64 voxels x 32 outputs
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int G = a.G;
    const int nbx = G / kPBX, nby = G / kPBY, nbz = G / kPBZ;
    const int ncb = (a.cout + 31) / 32, nch = a.cin / 32;
    // bricks per XCD (the brick count is a multiple of 8) and units per XCD
    const int bx = (int)(a.V / (kPBX * kPBY * kPBZ) / 8);
    const int ux = bx * ncb;
    const int xcd = (int)(blockIdx.x % 8);
    const int u0 = (int)(blockIdx.x / 8) * per, u1 = min(ux, u0 + per);
    if (u0 >= u1) return;
    const int kg = lane >> 4, lc = lane & 15;
    struct Unit {
        int x0, y0, z0, bs, cb;
    };
    auto unit = [&](int u) -> Unit {
        const int cb = u / bx, id = xcd * bx + u % bx;
        Unit w;
        w.x0 = __builtin_amdgcn_readfirstlane((id % nbx) * kPBX);
        w.y0 = __builtin_amdgcn_readfirstlane(((id / nbx) % nby) * kPBY);
        w.z0 = __builtin_amdgcn_readfirstlane(((id / (nbx * nby)) % nbz) * kPBZ);
        w.bs = __builtin_amdgcn_readfirstlane(id / (nbx * nby * nbz));
        w.cb = __builtin_amdgcn_readfirstlane(cb);
        return w;
    };
    // halo load u of a brick's chunk at channel c0: 64 consecutive threads
    // take 16 consecutive halo voxels x 4 channel groups; lanes past the halo
    // redo its last voxel, lanes outside the grid load a clamped voxel and
    // store zeros
    auto halo_at = [&](const Unit& w, int u, int& h, int& grp, unsigned& keep, int& xc, int& yc,
                       int& zc) {
        const int q = t + u * 512;
        h = min((q >> 6) * 16 + (q & 15), kPH - 1);
        grp = (q >> 4) & 3;
        const int hx = h % kPHX, hy = (h / kPHX) % kPHY, hz = h / (kPHX * kPHY);
        const int x = w.x0 + hx - 1, y = w.y0 + hy - 1, z = w.z0 + hz - 1;
        keep = (x >= 0 && x < G && y >= 0 && y < G && z >= 0 && z < G) ? ~0u : 0u;
        xc = min(max(x, 0), G - 1);
        yc = min(max(y, 0), G - 1);
        zc = min(max(z, 0), G - 1);
    };
    auto halo_load = [&](const Unit& w, int c, int u) -> uint4 {
        int h, grp, xc, yc, zc;
        unsigned keep;
        halo_at(w, u, h, grp, keep, xc, yc, zc);
        if (c * 32 < a.upc) {
            // an upsampled channel chunk: the parent voxel
            const int Gh = G >> 1;
            const int64_t pv = (((int64_t)w.bs * Gh + (zc >> 1)) * Gh + (yc >> 1)) * Gh + (xc >> 1);
            return *reinterpret_cast<const uint4*>(a.up + pv * a.upp + a.upo + c * 32 + grp * 8);
        }
        const int64_t gv = (((int64_t)w.bs * G + zc) * G + yc) * G + xc;
        return *reinterpret_cast<const uint4*>(a.in + gv * a.ip + a.io + c * 32 + grp * 8);
    };
    auto halo_store = [&](const Unit& w, int u, uint4 v) {
        int h, grp, xc, yc, zc;
        unsigned keep;
        halo_at(w, u, h, grp, keep, xc, yc, zc);
        v.x &= keep;
        v.y &= keep;
        v.z &= keep;
        v.w &= keep;
        *reinterpret_cast<uint4*>(&halo[grp][h]) = v;
    };
    // weight load u of chunk c for output block cb: element r of the chunk's
    // 27 x 4 x 32 run in the brick order holds offset r / 128, channel group
    // (r / 32) % 4, output cb 32 + r % 32 (lanes past the run redo its last
    // element)
    auto wts_load = [&](int cb, int c, int u) -> uint4 {
        const int r = min(t + u * 512, kPWts - 1);
        return a.wp[(int64_t)(cb * nch + c) * kPWts + r];
    };
    auto wts_store = [&](int u, uint4 v) {
        const int r = min(t + u * 512, kPWts - 1);
        *reinterpret_cast<uint4*>(&wl[r / 128][(r >> 5) & 3][r & 31]) = v;
    };
    // this lane's halo row 0 (output row -1, column lc) of its plane
    const int hv0 = (wave + 1) * kPHY * kPHX + lc + 1;
    // halo rows -1 .. 4 of this lane's plane shifted by (dz, dx) = (pl - 1,
    // dx - 1): row r serves output row mt at dy index r - mt
    auto loadA6 = [&](int g, bf16x8 (&A)[6]) {
        const int dh = (g / 3 - 1) * kPHY * kPHX + g % 3 - 1;
#pragma unroll
        for (int r = 0; r < 6; r++) A[r] = halo[kg][hv0 + r * kPHX + dh];
    };
    auto loadB = [&](int off, bf16x8 (&B)[2]) {
#pragma unroll
        for (int nt = 0; nt < 2; nt++) B[nt] = wl[off][kg][nt * 16 + lc];
    };
    uint4 hr[kPSPT], wr[kPWPT];
    {
        const Unit w = unit(u0);
#pragma unroll
        for (int u = 0; u < kPSPT; u++) hr[u] = halo_load(w, 0, u);
#pragma unroll
        for (int u = 0; u < kPWPT; u++) wr[u] = wts_load(w.cb, 0, u);
#pragma unroll
        for (int u = 0; u < kPSPT; u++) halo_store(w, u, hr[u]);
#pragma unroll
        for (int u = 0; u < kPWPT; u++) wts_store(u, wr[u]);
    }
    __syncthreads();
    // the 2 x 2 x 2 means of unit w's outputs, from the epilogue slots of
    // waves 2p and 2p + 1: wave p < 4 takes coarse plane p, lane: coarse voxel
    // lane / 4 (x fastest), channel group lane % 4; summed in the order dz,
    // dy, dx like k_pool_fwd.  Run by the waves after a barrier that follows
    // the unit's epilogue, before any slot is rewritten.
    auto pool_means = [&](const Unit& w) {
        if (wave >= 4) return;
        const int cv = lane >> 2, grp = lane & 3, cx = cv & 7, cy = cv >> 3;
        const int co = w.cb * 32 + grp * 8;
        float sum[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int d = 0; d < 8; d++) {
            const int m = (2 * cy + ((d >> 1) & 1)) * 16 + 2 * cx + (d & 1);
            const bf16x8 v =
                *reinterpret_cast<const bf16x8*>(&ep[2 * wave + (d >> 2)][m * 32 + grp * 8]);
#pragma unroll
            for (int e = 0; e < 8; e++) sum[e] += (float)v[e];
        }
        bf16x8 o;
#pragma unroll
        for (int e = 0; e < 8; e++) o[e] = (bf16)(sum[e] * 0.125f);
        const int Gh = G >> 1;
        const int64_t pv =
            (((int64_t)w.bs * Gh + (w.z0 >> 1) + wave) * Gh + (w.y0 >> 1) + cy) * Gh + (w.x0 >> 1) + cx;
        if (co < a.cout) *reinterpret_cast<bf16x8*>(a.pool + pv * a.pp + co) = o;
    };
    // a unit whose means are still to be written: they are formed at the
    // next barrier pair (the next item's end), after its epilogue
    bool pend = false;
    Unit wpend = unit(u0);
    for (int un = u0; un < u1; un++) {
        const Unit w = unit(un);
        const Unit wn = unit(min(un + 1, u1 - 1));
        f32x4 acc[4][2];
#pragma unroll
        for (int mt = 0; mt < 4; mt++)
#pragma unroll
            for (int nt = 0; nt < 2; nt++) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int c = 0; c < nch; c++) {
            // the next item: this unit's next chunk, or the next unit's first
            const bool more = c + 1 < nch, next = more || un + 1 < u1;
            const Unit& wx = more ? w : wn;
            const int cx = more ? c + 1 : 0;
            const bool new_w = next && (nch > 1 || wx.cb != w.cb);
            if (next) {
#pragma unroll
                for (int u = 0; u < kPSPT; u++) hr[u] = halo_load(wx, cx, u);
            }
            if (new_w) {
#pragma unroll
                for (int u = 0; u < kPWPT; u++) wr[u] = wts_load(wx.cb, cx, u);
            }
            // 27 steps: nine (dz, dx) groups of three dy offsets, offset
            // (dz, dy, dx) being weight row (dz + 1) 9 + (dy + 1) 3 + dx + 1;
            // a group's six halo rows are read one group ahead, the weights
            // two steps ahead
            auto step_off = [](int st) { return st / 9 * 9 + st % 3 * 3 + st / 3 % 3; };
            bf16x8 A[6], Bq[3][2];
            loadA6(0, A);
            loadB(step_off(0), Bq[0]);
            loadB(step_off(1), Bq[1]);
#pragma unroll
            for (int g = 0; g < 9; g++) {
                bf16x8 An[6];
#pragma unroll
                for (int dy = 0; dy < 3; dy++) {
                    const int st = g * 3 + dy;
                    if (st + 2 < 27) loadB(step_off(st + 2), Bq[(st + 2) % 3]);
                    if (dy == 0 && g < 8) loadA6(g + 1, An);
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int mt = 0; mt < 4; mt++)
#pragma unroll
                        for (int nt = 0; nt < 2; nt++)
                            acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                A[mt + dy], Bq[st % 3][nt], acc[mt][nt], 0, 0, 0);
                }
                if (g < 8) {
#pragma unroll
                    for (int r = 0; r < 6; r++) A[r] = An[r];
                }
            }
            if (next) {
                __syncthreads();  // no wave still reads this item's halo or weights
                if (pend) {
                    pool_means(wpend);
                    pend = false;
                }
#pragma unroll
                for (int u = 0; u < kPSPT; u++) halo_store(wx, u, hr[u]);
                if (new_w) {
#pragma unroll
                    for (int u = 0; u < kPWPT; u++) wts_store(u, wr[u]);
                }
                __syncthreads();
            }
        }
        // epilogue through this wave's LDS slot: C layout (lane holds rows
        // (lane / 16) 4 + i, column lane % 16) to voxel-major rows of 32
        // outputs, then 16-byte stores of eight outputs each
        // means still pending (no barrier pair since their epilogue): form
        // them now, between two barriers, before the slots are rewritten
        if (pend) {
            __syncthreads();
            pool_means(wpend);
            pend = false;
            __syncthreads();
        }
        bf16* ew = &ep[wave][0];
#pragma unroll
        for (int nt = 0; nt < 2; nt++) {
            const int col = nt * 16 + lc, co = w.cb * 32 + col;
            const float bias = a.bias && co < a.cout ? a.bias[co] : 0.0f;
#pragma unroll
            for (int mt = 0; mt < 4; mt++)
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    float val = acc[mt][nt][i] + bias;
                    if (a.relu) val = fmaxf(val, 0.0f);
                    ew[(mt * 16 + kg * 4 + i) * 32 + col] = (bf16)val;
                }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int p = 0; p < 4; p++) {
            const int idx = p * 64 + lane, m = idx >> 2, part = idx & 3;
            const int co = w.cb * 32 + part * 8;
            if (co >= a.cout) continue;  // cout is a multiple of 8
            bf16x8 v = *reinterpret_cast<const bf16x8*>(&ew[m * 32 + part * 8]);
            const int64_t vox =
                (((int64_t)w.bs * G + w.z0 + wave) * G + w.y0 + (m >> 4)) * G + w.x0 + (m & 15);
            if (a.mk) {
                const bf16x8 y = *reinterpret_cast<const bf16x8*>(a.mk + vox * a.mkp + a.mko + co);
#pragma unroll
                for (int e = 0; e < 8; e++)
                    if (!((float)y[e] > 0.0f)) v[e] = (bf16)0.0f;
            }
            *reinterpret_cast<bf16x8*>(a.out + vox * a.op + a.oo + co) = v;
        }
        if (a.pool) {
            pend = true;
            wpend = w;
        }
    }
    if (pend) {
        __syncthreads();
        pool_means(wpend);
    }
}

// The first layer (8 input channels) on the same bricks and schedule: one
// 32-wide MFMA step takes four offsets x 8 channels (lane group kg holds
// offset 4 s + kg), 7 steps for the 27 offsets, the 28th a zero weight row
// (its A lanes read offset 26, a finite value).  Halo 17 KB, weights 14 KB,
// at most 128 registers: two workgroups (16 waves) share a CU, whose other
// workgroup's waves cover a step's LDS latency.
constexpr int kP8Steps = 7;
constexpr int kP8Wts = kP8Steps * 4 * 32;     // 16-byte weight elements per block
constexpr int kP8SPT = (kPH + 511) / 512;     // halo loads per thread: 3
constexpr int kP8WPT = (kP8Wts + 511) / 512;  // weight loads per thread: 2

__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4)))
k_conv_p8(ConvArgs a, int per) {
    __shared__ bf16x8 halo[kPH];
    __shared__ bf16x8 wl[kP8Steps][4][32];
    __shared__ __align__(16) bf16 ep[8][64 * 32];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int G = a.G;
    const int nbx = G / kPBX, nby = G / kPBY, nbz = G / kPBZ;
    const int ncb = (a.cout + 31) / 32;
    const int bx = (int)(a.V / (kPBX * kPBY * kPBZ) / 8);
    const int ux = bx * ncb;
    const int xcd = (int)(blockIdx.x % 8);
    const int u0 = (int)(blockIdx.x / 8) * per, u1 = min(ux, u0 + per);
    if (u0 >= u1) return;
    const int kg = lane >> 4, lc = lane & 15;
    struct Unit {
        int x0, y0, z0, bs, cb;
    };
    auto unit = [&](int u) -> Unit {
        const int cb = u / bx, id = xcd * bx + u % bx;
        Unit w;
        w.x0 = __builtin_amdgcn_readfirstlane((id % nbx) * kPBX);
        w.y0 = __builtin_amdgcn_readfirstlane(((id / nbx) % nby) * kPBY);
        w.z0 = __builtin_amdgcn_readfirstlane(((id / (nbx * nby)) % nbz) * kPBZ);
        w.bs = __builtin_amdgcn_readfirstlane(id / (nbx * nby * nbz));
        w.cb = __builtin_amdgcn_readfirstlane(cb);
        return w;
    };
    // halo voxel q = t + 512 u (the last ones redone); outside the grid a
    // clamped voxel is loaded and zeros stored
    auto halo_at = [&](const Unit& w, int u, int& h, unsigned& keep) -> int64_t {
        h = min(t + u * 512, kPH - 1);
        const int hx = h % kPHX, hy = (h / kPHX) % kPHY, hz = h / (kPHX * kPHY);
        const int x = w.x0 + hx - 1, y = w.y0 + hy - 1, z = w.z0 + hz - 1;
        keep = (x >= 0 && x < G && y >= 0 && y < G && z >= 0 && z < G) ? ~0u : 0u;
        const int xc = min(max(x, 0), G - 1), yc = min(max(y, 0), G - 1),
                  zc = min(max(z, 0), G - 1);
        return (((int64_t)w.bs * G + zc) * G + yc) * G + xc;
    };
    auto halo_load = [&](const Unit& w, int u) -> uint4 {
        int h;
        unsigned keep;
        const int64_t gv = halo_at(w, u, h, keep);
        return *reinterpret_cast<const uint4*>(a.in + gv * a.ip + a.io);
    };
    auto halo_store = [&](const Unit& w, int u, uint4 v) {
        int h;
        unsigned keep;
        (void)halo_at(w, u, h, keep);
        v.x &= keep;
        v.y &= keep;
        v.z &= keep;
        v.w &= keep;
        *reinterpret_cast<uint4*>(&halo[h]) = v;
    };
    // weight element r of block cb: step r / 128, lane group (r / 32) % 4,
    // output cb 32 + r % 32
    auto wts_load = [&](int cb, int u) -> uint4 {
        const int r = min(t + u * 512, kP8Wts - 1);
        return a.wp[(int64_t)cb * kP8Wts + r];
    };
    auto wts_store = [&](int u, uint4 v) {
        const int r = min(t + u * 512, kP8Wts - 1);
        *reinterpret_cast<uint4*>(&wl[r / 128][(r >> 5) & 3][r & 31]) = v;
    };
    // this lane's halo index of step s, row mt: its voxel (lc, mt, wave)
    // shifted by offset min(4 s + kg, 26)
    const int hv0 = ((wave + 1) * kPHY + 1) * kPHX + lc + 1;
    auto loadA = [&](int s, bf16x8 (&A)[4]) {
        const int off = min(4 * s + kg, 26);
        const int dh = ((off / 9 - 1) * kPHY + (off / 3) % 3 - 1) * kPHX + off % 3 - 1;
#pragma unroll
        for (int mt = 0; mt < 4; mt++) A[mt] = halo[hv0 + mt * kPHX + dh];
    };
    auto loadB = [&](int s, bf16x8 (&B)[2]) {
#pragma unroll
        for (int nt = 0; nt < 2; nt++) B[nt] = wl[s][kg][nt * 16 + lc];
    };
    uint4 hr[kP8SPT], wr[kP8WPT];
    {
        const Unit w = unit(u0);
#pragma unroll
        for (int u = 0; u < kP8SPT; u++) hr[u] = halo_load(w, u);
#pragma unroll
        for (int u = 0; u < kP8WPT; u++) wr[u] = wts_load(w.cb, u);
#pragma unroll
        for (int u = 0; u < kP8SPT; u++) halo_store(w, u, hr[u]);
#pragma unroll
        for (int u = 0; u < kP8WPT; u++) wts_store(u, wr[u]);
    }
    __syncthreads();
    for (int un = u0; un < u1; un++) {
        const Unit w = unit(un);
        const bool next = un + 1 < u1;
        const Unit wn = unit(next ? un + 1 : un);
        const bool new_w = next && wn.cb != w.cb;
        if (next) {
#pragma unroll
            for (int u = 0; u < kP8SPT; u++) hr[u] = halo_load(wn, u);
        }
        if (new_w) {
#pragma unroll
            for (int u = 0; u < kP8WPT; u++) wr[u] = wts_load(wn.cb, u);
        }
        f32x4 acc[4][2];
#pragma unroll
        for (int mt = 0; mt < 4; mt++)
#pragma unroll
            for (int nt = 0; nt < 2; nt++) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int st = 0; st < kP8Steps; st++) {
            bf16x8 A[4], B[2];
            loadA(st, A);
            loadB(st, B);
#pragma unroll
            for (int mt = 0; mt < 4; mt++)
#pragma unroll
                for (int nt = 0; nt < 2; nt++)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mt], B[nt],
                                                                          acc[mt][nt], 0, 0, 0);
        }
        if (next) {
            __syncthreads();  // no wave still reads this unit's halo or weights
#pragma unroll
            for (int u = 0; u < kP8SPT; u++) halo_store(wn, u, hr[u]);
            if (new_w) {
#pragma unroll
                for (int u = 0; u < kP8WPT; u++) wts_store(u, wr[u]);
            }
            __syncthreads();
        }
        // epilogue through this wave's LDS slot, as in k_conv_p
        bf16* ew = &ep[wave][0];
#pragma unroll
        for (int nt = 0; nt < 2; nt++) {
            const int col = nt * 16 + lc, co = w.cb * 32 + col;
            const float bias = a.bias && co < a.cout ? a.bias[co] : 0.0f;
#pragma unroll
            for (int mt = 0; mt < 4; mt++)
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    float val = acc[mt][nt][i] + bias;
                    if (a.relu) val = fmaxf(val, 0.0f);
                    ew[(mt * 16 + kg * 4 + i) * 32 + col] = (bf16)val;
                }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int p = 0; p < 4; p++) {
            const int idx = p * 64 + lane, m = idx >> 2, part = idx & 3;
            const int co = w.cb * 32 + part * 8;
            if (co >= a.cout) continue;
            const uint4 v = *reinterpret_cast<const uint4*>(&ew[m * 32 + part * 8]);
            const int64_t vox =
                (((int64_t)w.bs * G + w.z0 + wave) * G + w.y0 + (m >> 4)) * G + w.x0 + (m & 15);
            *reinterpret_cast<uint4*>(a.out + vox * a.op + a.oo + co) = v;
        }
    }
}

hipError_t conv_fwd(const ConvArgs& a, hipStream_t s) {
    const int G = a.G;
    if ((a.upc || a.pool || a.mk) &&
        !(a.ks == 3 && a.cin % 32 == 0 && a.upc % 32 == 0 && G % 16 == 0 && a.wp &&
          a.pp % 8 == 0 && a.mkp % 8 == 0 && a.mko % 8 == 0))
        return hipErrorInvalidValue;  // only the brick kernel reads upsampled channels, pools
                                      // and masks
    if (a.ks == 3 && a.cin == 8 && G % 16 == 0 && a.wp && a.cout % 8 == 0 && a.op % 8 == 0 &&
        a.oo % 8 == 0 && a.ip % 8 == 0 && a.io % 8 == 0) {
        // the first layer on the same bricks
        const int64_t nb = a.V / (kPBX * kPBY * kPBZ);
        const int64_t ux = nb / 8 * ((a.cout + 31) / 32);
        if (nb % 8 == 0 && ux <= INT32_MAX) {
            // 64 KB of LDS: two workgroups per CU
            const int64_t wgs = std::min<int64_t>(ux, 2 * kPWGPerXcd);
            const int per = (int)((ux + wgs - 1) / wgs);
            hipLaunchKernelGGL(k_conv_p8, dim3((unsigned)(8 * wgs)), dim3(512), 0, s, a, per);
            return hipGetLastError();
        }
    }
    if (a.ks == 3 && a.cin % 32 == 0 && G % 16 == 0 && a.wp && a.cout % 8 == 0 &&
        a.op % 8 == 0 && a.oo % 8 == 0) {
        // 16 x 4 x 8 bricks; their count, B G^3 / 512, is a multiple of 8
        const int64_t nb = a.V / (kPBX * kPBY * kPBZ);
        const int64_t ux = nb / 8 * ((a.cout + 31) / 32);
        if (nb % 8 == 0 && ux <= INT32_MAX) {
            const int64_t wgs = std::min<int64_t>(ux, kPWGPerXcd);
            const int per = (int)((ux + wgs - 1) / wgs);
            hipLaunchKernelGGL(k_conv_p, dim3((unsigned)(8 * wgs)), dim3(512), 0, s, a, per);
            return hipGetLastError();
        }
    }
    if (a.upc || a.pool || a.mk) return hipErrorInvalidValue;
    if (a.ks == 3 && a.cin % 32 == 0 && G >= 8 && (G & (G - 1)) == 0) {
        // bricks of 256 voxels: 16 x 8 x 2, or 8 x 8 x 4 on an 8^3 grid
        const int BX = G >= 16 ? 16 : 8, BY = 8, BZ = 256 / (BX * BY);
        const int64_t G3 = (int64_t)G * G * G;
        const int64_t nsamp = a.V / G3;
        const dim3 grid((unsigned)(nsamp * (G3 / 256)), (unsigned)((a.cout + 63) / 64));
        if (a.cout <= 16)
            hipLaunchKernelGGL(k_conv_lds<1>, grid, dim3(256), 0, s, a, BX, BY, BZ);
        else if (a.cout <= 32)
            hipLaunchKernelGGL(k_conv_lds<2>, grid, dim3(256), 0, s, a, BX, BY, BZ);
        else
            hipLaunchKernelGGL(k_conv_lds<4>, grid, dim3(256), 0, s, a, BX, BY, BZ);
        return hipGetLastError();
    }
    const dim3 grid(nblocks(a.V, 256), (unsigned)((a.cout + 63) / 64));
    if (a.cout <= 16)
        hipLaunchKernelGGL(k_conv_fwd<1>, grid, dim3(256), 0, s, a);
    else if (a.cout <= 32)
        hipLaunchKernelGGL(k_conv_fwd<2>, grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_conv_fwd<4>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Weight and bias gradient
// ---------------------------------------------------------------------------
// dW[co][k] = sum_v D[v][co] X[v + off(k)][ci(k)] and db[co] = sum_v D[v][co]:
// an MFMA product with the voxels as the reduction dimension.  The bias is
// the extra column k = K of X, equal to 1 on every voxel.  A workgroup owns
// a COT x KN tile (output channels x k) and one split of the voxels, which
// it walks in chunks of CV voxels.  Each chunk is staged transposed in LDS
// (channel-major rows of CV voxels): a thread gathers 8-voxel x 8-channel
// blocks with 16-byte loads, transposes them in registers and writes 8 rows
// of 16 bytes each.  Each wave then multiplies an (MT x 16) x (NT x 16)
// block, reusing its MT + NT fragments for MT x NT MFMAs per 32 voxels.
// The next chunk's loads are in flight during the current chunk's
// products, so a longer chunk hides more of their latency.
struct WgradArgs {
    const bf16* d;  // gradient of the pre-activation output, [V][dp]
    int dp, doff, cout;
    const bf16* in;  // convolution input
    int ip, io, cin;
    const bf16* up = nullptr;  // input channels [0, upc) at half resolution, as in ConvArgs
    int upp = 0, upo = 0, upc = 0;
    int G;
    int64_t V, vsplit;
    int kp2;      // k extent of the partial buffer (multiple of KN, > 27 cin)
    float* part;  // [splits][cout][kp2]
};

__device__ __forceinline__ void transpose_store8(const bf16x8 (&r)[8], bf16* row0, int pitch) {
#pragma unroll
    for (int j = 0; j < 8; j++) {
        bf16x8 o;
#pragma unroll
        for (int i = 0; i < 8; i++) o[i] = r[i][j];
        *reinterpret_cast<bf16x8*>(row0 + j * pitch) = o;
    }
}

template <int MT, int NT, int WM, int WN, int CV>
__global__ void __launch_bounds__(256) k_wgrad(WgradArgs a) {
    constexpr int COT = 16 * MT * WM, KN = 16 * NT * WN, LP = CV + 8;
    constexpr int VG = CV / 8;                          // voxel groups per chunk
    constexpr int XPT = (KN / 8 * VG + 255) / 256;      // input blocks per thread
    constexpr int DPT = (COT / 8 * VG + 255) / 256;     // gradient blocks per thread
    static_assert(WM * WN == 4, "four waves");
    static_assert(CV % 32 == 0, "whole MFMA k-steps per chunk");
    __shared__ __align__(16) bf16 sD[COT][LP];
    __shared__ __align__(16) bf16 sX[KN][LP];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int k0 = blockIdx.x * KN, co0 = blockIdx.y * COT;
    const int64_t vs = (int64_t)blockIdx.z * a.vsplit;
    const int64_t ve = min(a.V, vs + a.vsplit);
    const int G = a.G;
    const int64_t G3 = (int64_t)G * G * G;
    const int K = 27 * a.cin;
    // staging blocks of this thread, the same for every chunk: block
    // b = t + 256 u covers k-group (or channel group) b / VG and voxel group
    // b % VG of the chunk; 8 consecutive k never straddle an offset or K, as
    // cin % 8 == 0
    int xg[XPT], xvg[XPT], xci[XPT], xdz[XPT], xdy[XPT], xdx[XPT];
    bool xon[XPT], xdat[XPT];
#pragma unroll
    for (int u = 0; u < XPT; u++) {
        const int bl = t + 256 * u;
        xon[u] = bl < KN / 8 * VG;
        xg[u] = bl / VG;
        xvg[u] = bl % VG;
        const int kk = k0 + xg[u] * 8;
        xdat[u] = xon[u] && kk < K;
        xci[u] = xdz[u] = xdy[u] = xdx[u] = 0;
        if (xdat[u]) {
            const int off = kk / a.cin;
            xci[u] = kk - off * a.cin;
            xdz[u] = off / 9 - 1;
            xdy[u] = (off / 3) % 3 - 1;
            xdx[u] = off % 3 - 1;
        }
    }
    int dg[DPT], dvg[DPT];
    bool don[DPT], ddat[DPT];
#pragma unroll
    for (int u = 0; u < DPT; u++) {
        const int bl = t + 256 * u;
        don[u] = bl < COT / 8 * VG;
        dg[u] = bl / VG;
        dvg[u] = bl % VG;
        ddat[u] = don[u] && co0 + dg[u] * 8 < a.cout;
    }
    // registers of one chunk's blocks; the next chunk's loads are in flight
    // while the current chunk is multiplied
    bf16x8 rX[XPT][8], rD[DPT][8];
    auto fetch = [&](int64_t vc) {
#pragma unroll
        for (int u = 0; u < XPT; u++) {
            const int64_t v0 = vc + xvg[u] * 8;
            if (xdat[u]) {
                int64_t b = v0 / G3;
                const int64_t r = v0 - b * G3;
                int z = (int)(r / ((int64_t)G * G)), y = (int)((r / G) % G), x = (int)(r % G);
#pragma unroll
                for (int i = 0; i < 8; i++) {
                    rX[u][i] = zero8();
                    const int z2 = z + xdz[u], y2 = y + xdy[u], x2 = x + xdx[u];
                    if (v0 + i < ve && z2 >= 0 && z2 < G && y2 >= 0 && y2 < G && x2 >= 0 &&
                        x2 < G) {
                        const int64_t nv = ((b * G + z2) * G + y2) * G + x2;
                        rX[u][i] = *reinterpret_cast<const bf16x8*>(a.in + nv * a.ip + a.io + xci[u]);
                    }
                    if (++x == G) {  // next voxel in x-fastest order
                        x = 0;
                        if (++y == G) {
                            y = 0;
                            if (++z == G) {
                                z = 0;
                                ++b;
                            }
                        }
                    }
                }
            } else {
                const bool bias = xon[u] && k0 + xg[u] * 8 == K;
#pragma unroll
                for (int i = 0; i < 8; i++) {
                    rX[u][i] = zero8();
                    if (bias && v0 + i < ve) rX[u][i][0] = (bf16)1.0f;  // bias column
                }
            }
        }
#pragma unroll
        for (int u = 0; u < DPT; u++) {
            const int64_t v0 = vc + dvg[u] * 8;
            const int co = co0 + dg[u] * 8;
#pragma unroll
            for (int i = 0; i < 8; i++)
                rD[u][i] = (ddat[u] && v0 + i < ve)
                               ? *reinterpret_cast<const bf16x8*>(a.d + (v0 + i) * a.dp + a.doff + co)
                               : zero8();
        }
    };
    f32x4 acc[MT][NT];
#pragma unroll
    for (int mt = 0; mt < MT; mt++)
#pragma unroll
        for (int nt = 0; nt < NT; nt++) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (vs < ve) fetch(vs);
    for (int64_t vc = vs; vc < ve; vc += CV) {
        __syncthreads();  // the previous chunk's fragments have been read
#pragma unroll
        for (int u = 0; u < XPT; u++)
            if (xon[u]) transpose_store8(rX[u], &sX[xg[u] * 8][xvg[u] * 8], LP);
#pragma unroll
        for (int u = 0; u < DPT; u++)
            if (don[u]) transpose_store8(rD[u], &sD[dg[u] * 8][dvg[u] * 8], LP);
        if (vc + CV < ve) fetch(vc + CV);
        __syncthreads();
#pragma unroll
        for (int s2 = 0; s2 < CV / 32; s2++) {
            const int vo = s2 * 32 + (lane >> 4) * 8;
            bf16x8 A[MT], Bf[NT];
#pragma unroll
            for (int mt = 0; mt < MT; mt++)
                A[mt] = *reinterpret_cast<const bf16x8*>(&sD[(wm * MT + mt) * 16 + (lane & 15)][vo]);
#pragma unroll
            for (int nt = 0; nt < NT; nt++)
                Bf[nt] = *reinterpret_cast<const bf16x8*>(&sX[(wn * NT + nt) * 16 + (lane & 15)][vo]);
#pragma unroll
            for (int mt = 0; mt < MT; mt++)
#pragma unroll
                for (int nt = 0; nt < NT; nt++)
                    acc[mt][nt] =
                        __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mt], Bf[nt], acc[mt][nt], 0, 0, 0);
        }
    }
    // C layout: lane holds rows (lane / 16) * 4 + i, column lane % 16
#pragma unroll
    for (int mt = 0; mt < MT; mt++)
#pragma unroll
        for (int nt = 0; nt < NT; nt++)
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int co = co0 + (wm * MT + mt) * 16 + (lane >> 4) * 4 + i;
                const int k = k0 + (wn * NT + nt) * 16 + (lane & 15);
                if (co < a.cout)
                    a.part[((int64_t)blockIdx.z * a.cout + co) * a.kp2 + k] = acc[mt][nt][i];
            }
}

// Brick form of the weight gradient, for G % 16 == 0 and cin, cout multiples
// of 32: dW[co][off][ci] = sum_v D[v][co] X[v + off][ci] with the voxels v
// of 16 x 4 x 4 bricks as the MFMA reduction dimension.  A workgroup of 8
// waves owns CI = 32 input channels (blockIdx.x), 32 output channels
// (blockIdx.y) and a run of bricks (blockIdx.z); the next brick's loads are
// in flight (in registers) while the current one is multiplied.  For each brick it stages,
// once, the gradient D transposed (32 channel rows of the 256 brick voxels)
// and the input's halo (18 x 6 x 6 voxels) transposed as channel rows of 16
// x positions, in three copies shifted by dx = -1, 0, 1, so that the 8
// consecutive voxels an MFMA lane takes start 16-byte aligned for every
// offset.  Each wave then accumulates up to four of the 27 offsets (wave w:
// offsets w, w + 8, w + 16, w + 24; offset 27 is the bias, a column of ones)
// for all of the brick's voxels: the halo, fetched once from memory, serves
// all 27 offsets, where the gathered form fetched it once per offset.
// Partial sums per brick run go to part[split] like k_wgrad's, and
// k_wgrad_reduce adds them in a fixed order (bit-reproducible).
constexpr int kGRows = 6 * 6;  // halo rows (y, z) of a 16 x 4 x 4 brick
// channel rows padded by 16 bytes: the 16 channels of an MFMA fragment then
// start 4 banks apart and read all 64 banks once
constexpr int kGXP = kGRows * 16 + 8;  // halo copy: bf16 per channel row
constexpr int kGDP = 256 + 8;          // D^T: bf16 per channel row

template <int CI>
__global__ void __launch_bounds__(512) k_wgrad_brick(WgradArgs a, int64_t per_split) {
    constexpr int NT = CI / 16;  // 16-channel column tiles
    __shared__ __align__(16) bf16 xs[3][CI][kGXP];
    __shared__ __align__(16) bf16 dT[32][kGDP];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int c0 = blockIdx.x * CI, co0 = blockIdx.y * 32;
    const int G = a.G;
    const int nbx = G / 16, nby = G / 4, nbz = G / 4;
    const int64_t nb = a.V / 256;
    const int64_t b0 = (int64_t)blockIdx.z * per_split, b1 = min(nb, b0 + per_split);
    const int kg = lane >> 4, lc = lane & 15;
    const bool bias_here = blockIdx.x == 0;
    // staging tasks: threads [0, 128) take 8 brick voxels x 8 output
    // channels of D, threads [128, 128 + 72 CI / 8) half a halo row (x
    // positions 8 g .. 8 g + 9 of its 18) of 8 input channels, for all three
    // shifted copies; the loads of the next brick are in flight during the
    // current brick's products
    const bool dtask = t < 128, xtask = !dtask && t < 128 + 2 * kGRows * (CI / 8);
    const int cg = t & 3, vg = t >> 2;  // D task
    const int xt = t - 128, row = xt / (2 * (CI / 8)), cgp = xt % (CI / 8),
              gx = (xt / (CI / 8)) & 1;  // halo task
    bf16x8 st[10];
    auto stage_load = [&](int64_t b) {
        const int bx = (int)(b % nbx), by = (int)((b / nbx) % nby),
                  bz = (int)((b / ((int64_t)nbx * nby)) % nbz);
        const int64_t bs = b / ((int64_t)nbx * nby * nbz);
        const int x0 = bx * 16, y0 = by * 4, z0 = bz * 4;
        if (dtask) {
            const int co = co0 + cg * 8;
#pragma unroll
            for (int i = 0; i < 8; i++) {
                const int vb = vg * 8 + i;
                const int64_t v =
                    ((bs * G + z0 + vb / 64) * G + y0 + (vb / 16) % 4) * G + x0 + vb % 16;
                st[i] = co < a.cout ? *reinterpret_cast<const bf16x8*>(a.d + v * a.dp + a.doff + co)
                                    : zero8();
            }
        } else if (xtask) {
            const int hy = row % 6, hz = row / 6;
            const int y = y0 + hy - 1, z = z0 + hz - 1;
            const bool rowin = y >= 0 && y < G && z >= 0 && z < G;
            const int zc = min(max(z, 0), G - 1), yc = min(max(y, 0), G - 1);
            // the row's first voxel and x stride; an upsampled channel chunk
            // reads the parent row at half resolution (x / 2)
            const bool upc = c0 < a.upc;
            const int Gh = G >> 1;
            const bf16* row_p =
                upc ? a.up + (((bs * Gh + (zc >> 1)) * Gh + (yc >> 1)) * Gh) * a.upp + a.upo + c0 +
                          cgp * 8
                    : a.in + (((bs * G + zc) * G + yc) * G) * a.ip + a.io + c0 + cgp * 8;
            const int xs = upc ? 1 : 0;
            const int64_t pitch = upc ? a.upp : a.ip;
#pragma unroll
            for (int e = 0; e < 10; e++) {
                const int x = x0 + gx * 8 + e - 1;
                st[e] = (rowin && x >= 0 && x < G)
                            ? *reinterpret_cast<const bf16x8*>(row_p + (int64_t)(x >> xs) * pitch)
                            : zero8();
            }
        }
    };
    auto stage_store = [&]() {
        if (dtask) {
            bf16x8 r[8];
#pragma unroll
            for (int i = 0; i < 8; i++) r[i] = st[i];
            transpose_store8(r, &dT[cg * 8][vg * 8], kGDP);
        } else if (xtask) {
            // copy s holds halo x position x' + s at x' (this task: x' in
            // [8 gx, 8 gx + 8), positions 8 gx + s .. held in st[s ..])
#pragma unroll
            for (int sh = 0; sh < 3; sh++) {
                bf16x8 r[8];
#pragma unroll
                for (int i = 0; i < 8; i++) r[i] = st[sh + i];
                transpose_store8(r, &xs[sh][cgp * 8][row * 16 + 8 * gx], kGXP);
            }
        }
    };
    f32x4 acc[4][2][NT];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int mt = 0; mt < 2; mt++)
#pragma unroll
            for (int nt = 0; nt < NT; nt++) acc[i][mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    // the bias column: ones in column 0
    bf16x8 ones;
#pragma unroll
    for (int j = 0; j < 8; j++) ones[j] = (bf16)(lc == 0 ? 1.0f : 0.0f);
    if (b0 < b1) stage_load(b0);
    for (int64_t b = b0; b < b1; b++) {
        __syncthreads();  // the previous brick's fragments have been read
        stage_store();
        __syncthreads();
        if (b + 1 < b1) stage_load(b + 1);
#pragma unroll 2
        for (int ks = 0; ks < 8; ks++) {
            // this lane's 8 voxels: brick voxels ks * 32 + kg * 8 ..
            const int vb = ks * 32 + kg * 8;
            const int xl = vb % 16, yl = (vb / 16) % 4, zl = vb / 64;
            bf16x8 A[2];
#pragma unroll
            for (int mt = 0; mt < 2; mt++)
                A[mt] = *reinterpret_cast<const bf16x8*>(&dT[mt * 16 + lc][vb]);
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int off = wave + 8 * i;
                if (off < 27) {
                    const int dz = off / 9 - 1, dy = (off / 3) % 3 - 1, dx = off % 3 - 1;
                    const int hrow = (zl + dz + 1) * 6 + (yl + dy + 1);
                    bf16x8 B[NT];
#pragma unroll
                    for (int nt = 0; nt < NT; nt++)
                        B[nt] = *reinterpret_cast<const bf16x8*>(
                            &xs[dx + 1][nt * 16 + lc][hrow * 16 + xl]);
#pragma unroll
                    for (int mt = 0; mt < 2; mt++)
#pragma unroll
                        for (int nt = 0; nt < NT; nt++)
                            acc[i][mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                A[mt], B[nt], acc[i][mt][nt], 0, 0, 0);
                } else if (off == 27 && bias_here) {
#pragma unroll
                    for (int mt = 0; mt < 2; mt++)
                        acc[i][mt][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            A[mt], ones, acc[i][mt][0], 0, 0, 0);
                }
            }
        }
    }
    // C layout: lane holds rows (lane / 16) * 4 + j (output channels),
    // column lane % 16 (input channel; the bias in column 0)
    const int K = 27 * a.cin;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const int off = wave + 8 * i;
        if (off > 27 || (off == 27 && !bias_here)) continue;
#pragma unroll
        for (int mt = 0; mt < 2; mt++)
#pragma unroll
            for (int nt = 0; nt < NT; nt++) {
                if (off == 27 && (nt != 0 || lc != 0)) continue;
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    const int co = co0 + mt * 16 + kg * 4 + j;
                    const int k = off == 27 ? K : off * a.cin + c0 + nt * 16 + lc;
                    if (co < a.cout)
                        a.part[((int64_t)blockIdx.z * a.cout + co) * a.kp2 + k] = acc[i][mt][nt][j];
                }
            }
    }
}

// voxels per staged chunk of the weight gradient
constexpr int kWgradChunk = 128;

// tile shape of the weight gradient for a layer with `cout` output channels
inline int wgrad_kn(int cout) { return cout <= 32 ? 256 : 128; }
inline int wgrad_cot(int cout) { return cout <= 32 ? 32 : (cout <= 64 ? 64 : 128); }
constexpr int kWgradBlocks = 1024;  // workgroups aimed at per layer
// the brick form runs one workgroup per CU (128 KB of LDS): one wave of them
constexpr int kWgradBrickBlocks = 256;

// voxel split of a layer's weight gradient: ~kWgradBlocks workgroups, splits
// of whole chunks; never more than kWgradBlocks / tiles splits
inline int64_t wgrad_vsplit(int64_t V, int tiles) {
    const int64_t want = std::max<int64_t>(1, (kWgradBlocks + tiles - 1) / tiles);
    const int64_t vs = (V + want - 1) / want;
    return std::max<int64_t>(kWgradChunk,
                             (vs + kWgradChunk - 1) / kWgradChunk * kWgradChunk);
}

hipError_t launch_wgrad(const WgradArgs& w, int tiles_k, int tiles_c, int64_t splits,
                        hipStream_t s) {
    const dim3 grid((unsigned)tiles_k, (unsigned)tiles_c, (unsigned)splits);
    if (w.cout <= 32)
        hipLaunchKernelGGL((k_wgrad<2, 4, 1, 4, kWgradChunk>), grid, dim3(256), 0, s, w);
    else if (w.cout <= 64)
        hipLaunchKernelGGL((k_wgrad<2, 4, 2, 2, kWgradChunk>), grid, dim3(256), 0, s, w);
    else
        hipLaunchKernelGGL((k_wgrad<4, 4, 2, 2, kWgradChunk>), grid, dim3(256), 0, s, w);
    return hipGetLastError();
}

// dW[co][k] (k < K) and db[co] (column K): fixed-order sums over the splits.
// A workgroup takes 64 consecutive outputs; its four waves sum a quarter of
// the splits each (in ascending order, eight loads in flight), and the four
// quarter sums are added in order: the same tree for every call.
__global__ void __launch_bounds__(256) k_wgrad_reduce(const float* __restrict__ part, int splits,
                                                      int cout, int kp2, int K,
                                                      float* __restrict__ dW,
                                                      float* __restrict__ db) {
    __shared__ float q[4][64];
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t i = (int64_t)blockIdx.x * 64 + l;
    const int64_t nW = (int64_t)cout * K;
    const bool on = i < nW + cout;
    const int co = !on ? 0 : (i < nW ? (int)(i / K) : (int)(i - nW));
    const int k = !on ? 0 : (i < nW ? (int)(i % K) : K);
    const int per = (splits + 3) / 4, z0 = w * per, z1 = min(splits, z0 + per);
    float s = 0.0f;
    if (on) {
        int z = z0;
        for (; z + 8 <= z1; z += 8) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; u++) v[u] = part[((int64_t)(z + u) * cout + co) * kp2 + k];
#pragma unroll
            for (int u = 0; u < 8; u++) s += v[u];
        }
        for (; z < z1; z++) s += part[((int64_t)z * cout + co) * kp2 + k];
    }
    q[w][l] = s;
    __syncthreads();
    if (w == 0 && on) {
        const float r = ((q[0][l] + q[1][l]) + q[2][l]) + q[3][l];
        if (i < nW) dW[i] = r;
        else db[co] = r;
    }
}

// ---------------------------------------------------------------------------
// Elementwise passes (8 channels per thread)
// ---------------------------------------------------------------------------
// out[v][c] (contiguous) = g[v][c] if y[v][c] > 0 else 0
__global__ void k_relu_bwd(const bf16* __restrict__ g, int gp, int go, const bf16* __restrict__ y,
                           int yp, int yo, int C, int64_t V, bf16* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c8 = C / 8;
    if (i >= V * c8) return;
    const int64_t v = i / c8;
    const int c = (int)(i % c8) * 8;
    const bf16x8 gv = *reinterpret_cast<const bf16x8*>(g + v * gp + go + c);
    const bf16x8 yv = *reinterpret_cast<const bf16x8*>(y + v * yp + yo + c);
    bf16x8 o;
#pragma unroll
    for (int j = 0; j < 8; j++) o[j] = ((float)yv[j] > 0.0f) ? gv[j] : (bf16)0.0f;
    *reinterpret_cast<bf16x8*>(out + v * C + c) = o;
}

// out (contiguous, grid G/2) = mean of the 2x2x2 children of in (grid G)
// Coarse voxel u = ((b H + Z) H + Y) H + X of a 2 x 2 x 2 level pair (fine
// edge G = 2 H), in 32-bit arithmetic (the launchers keep B G^3 C / 8 below
// 2^31); `v0` is its first fine voxel, the others at + dz G^2 + dy G + dx.
struct Coarse {
    uint32_t u, v0;
};
__device__ inline Coarse coarse_of(uint32_t u, int G) {
    const uint32_t H = (uint32_t)G / 2;
    const uint32_t u2 = u / H, X = u - u2 * H;
    const uint32_t u3 = u2 / H, Y = u2 - u3 * H;
    const uint32_t b = u3 / H, Z = u3 - b * H;
    return {u, ((b * (uint32_t)G + 2 * Z) * (uint32_t)G + 2 * Y) * (uint32_t)G + 2 * X};
}
__device__ inline uint32_t child(uint32_t v0, int d, int G) {
    return v0 + (uint32_t)(d >> 2) * (uint32_t)G * (uint32_t)G + (uint32_t)((d >> 1) & 1) * (uint32_t)G +
           (uint32_t)(d & 1);
}

__global__ void k_pool_fwd(const bf16* __restrict__ in, int ip, int io, int C, int G, int B,
                           bf16* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int H = G / 2, c8 = C / 8;
    const int64_t n = (int64_t)B * H * H * H * c8;
    if (i >= n) return;
    const uint32_t i32 = (uint32_t)i;
    const int c = (int)(i32 % (uint32_t)c8) * 8;
    const Coarse q = coarse_of(i32 / (uint32_t)c8, G);
    bf16x8 x[8];
#pragma unroll
    for (int d = 0; d < 8; d++)
        x[d] = *reinterpret_cast<const bf16x8*>(in + (int64_t)child(q.v0, d, G) * ip + io + c);
    float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int d = 0; d < 8; d++)
#pragma unroll
        for (int j = 0; j < 8; j++) s[j] += (float)x[d][j];
    bf16x8 o;
#pragma unroll
    for (int j = 0; j < 8; j++) o[j] = (bf16)(s[j] * 0.125f);
    *reinterpret_cast<bf16x8*>(out + (int64_t)q.u * C + c) = o;
}

// out[v][c] (contiguous, grid G) = a[v][c] + gp[parent(v)][c] / 8
// one thread per coarse voxel and 8 channels: out = a + g / 8 at its
// children, then through the ReLU whose output is y (kept where y > 0)
__global__ void k_pool_bwd_add(const bf16* __restrict__ a, int ap, int ao,
                               const bf16* __restrict__ gpar, int C, int G, int B,
                               const bf16* __restrict__ y, int yp, int yo,
                               bf16* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c8 = C / 8, H = G / 2;
    const int64_t n = (int64_t)B * H * H * H * c8;
    if (i >= n) return;
    const uint32_t i32 = (uint32_t)i;
    const int c = (int)(i32 % (uint32_t)c8) * 8;
    const Coarse q = coarse_of(i32 / (uint32_t)c8, G);
    const bf16x8 gv = *reinterpret_cast<const bf16x8*>(gpar + (int64_t)q.u * C + c);
    bf16x8 av[8], yv[8];
#pragma unroll
    for (int d = 0; d < 8; d++) {
        const int64_t v = child(q.v0, d, G);
        av[d] = *reinterpret_cast<const bf16x8*>(a + v * ap + ao + c);
        yv[d] = *reinterpret_cast<const bf16x8*>(y + v * yp + yo + c);
    }
#pragma unroll
    for (int d = 0; d < 8; d++) {
        bf16x8 o;
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const bf16 gsum = (bf16)((float)av[d][j] + 0.125f * (float)gv[j]);
            o[j] = (float)yv[d][j] > 0.0f ? gsum : (bf16)0.0f;
        }
        *reinterpret_cast<bf16x8*>(out + (int64_t)child(q.v0, d, G) * C + c) = o;
    }
}

// out[v][oo + c] (grid G) = in[parent(v)][c] (contiguous, grid G/2)
// one thread per coarse voxel and 8 channels: its value to the 8 children
__global__ void k_up_fwd(const bf16* __restrict__ in, int C, int G, int B, bf16* __restrict__ out,
                         int op, int oo) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c8 = C / 8, H = G / 2;
    const int64_t n = (int64_t)B * H * H * H * c8;
    if (i >= n) return;
    const uint32_t i32 = (uint32_t)i;
    const int c = (int)(i32 % (uint32_t)c8) * 8;
    const Coarse q = coarse_of(i32 / (uint32_t)c8, G);
    const bf16x8 x = *reinterpret_cast<const bf16x8*>(in + (int64_t)q.u * C + c);
#pragma unroll
    for (int d = 0; d < 8; d++)
        *reinterpret_cast<bf16x8*>(out + (int64_t)child(q.v0, d, G) * op + oo + c) = x;
}

// out[u][c] (contiguous, grid G/2) = sum of g over the 2x2x2 children of u
// one thread per coarse voxel and 8 channels: the sum over its children,
// then through the ReLU whose output is y (kept where y > 0)
__global__ void k_up_bwd(const bf16* __restrict__ g, int gp, int go, int C, int G, int B,
                         const bf16* __restrict__ y, int yp, int yo, bf16* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int H = G / 2, c8 = C / 8;
    const int64_t n = (int64_t)B * H * H * H * c8;
    if (i >= n) return;
    const uint32_t i32 = (uint32_t)i;
    const int c = (int)(i32 % (uint32_t)c8) * 8;
    const Coarse q = coarse_of(i32 / (uint32_t)c8, G);
    bf16x8 x[8];
#pragma unroll
    for (int d = 0; d < 8; d++)
        x[d] = *reinterpret_cast<const bf16x8*>(g + (int64_t)child(q.v0, d, G) * gp + go + c);
    float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int d = 0; d < 8; d++)
#pragma unroll
        for (int j = 0; j < 8; j++) s[j] += (float)x[d][j];
    const bf16x8 yv = *reinterpret_cast<const bf16x8*>(y + (int64_t)q.u * yp + yo + c);
    bf16x8 o;
#pragma unroll
    for (int j = 0; j < 8; j++) o[j] = (float)yv[j] > 0.0f ? (bf16)s[j] : (bf16)0.0f;
    *reinterpret_cast<bf16x8*>(out + (int64_t)q.u * C + c) = o;
}

// y[v] = sum_c w[c] d[v][c] + b (32 channels)
__global__ void k_head_fwd(const bf16* __restrict__ d, const float* __restrict__ w, int64_t V,
                           float* __restrict__ y) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    float s = w[32];
#pragma unroll
    for (int c8 = 0; c8 < 4; c8++) {
        const bf16x8 x = *reinterpret_cast<const bf16x8*>(d + v * 32 + c8 * 8);
#pragma unroll
        for (int j = 0; j < 8; j++) s += w[c8 * 8 + j] * (float)x[j];
    }
    y[v] = s;
}

// block sums in a fixed tree order
__device__ float block_sum256(float v, float* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const float r = sh[0];
    __syncthreads();
    return r;
}

// g[v][c] = dy[v] w[c]; partials of dL/dw[c] = sum dy d[v][c] and dL/db
__global__ void __launch_bounds__(256) k_head_bwd(const float* __restrict__ dy,
                                                  const bf16* __restrict__ d,
                                                  const float* __restrict__ w, int64_t V,
                                                  bf16* __restrict__ g, float* __restrict__ part) {
    __shared__ float sh[256];
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float dv = 0.0f;
    float x[32];
    if (v < V) {
        dv = dy[v];
#pragma unroll
        for (int c8 = 0; c8 < 4; c8++) {
            const bf16x8 xv = *reinterpret_cast<const bf16x8*>(d + v * 32 + c8 * 8);
            bf16x8 o;
#pragma unroll
            for (int j = 0; j < 8; j++) {
                x[c8 * 8 + j] = (float)xv[j];
                // through d1b's ReLU: kept where its output is positive
                o[j] = x[c8 * 8 + j] > 0.0f ? (bf16)(dv * w[c8 * 8 + j]) : (bf16)0.0f;
            }
            *reinterpret_cast<bf16x8*>(g + v * 32 + c8 * 8) = o;
        }
    } else {
#pragma unroll
        for (int c = 0; c < 32; c++) x[c] = 0.0f;
    }
    // the block's 33 sums (dy x per channel, and dy): a butterfly within
    // each wave, then the four waves' sums in order (fixed, so the result is
    // reproducible)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < 33; c++) {
        float v = c < 32 ? dv * x[c] : dv;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) sh[wave * 33 + c] = v;
    }
    __syncthreads();
    if (threadIdx.x < 33)
        part[(int64_t)blockIdx.x * 33 + threadIdx.x] =
            ((sh[threadIdx.x] + sh[33 + threadIdx.x]) + sh[66 + threadIdx.x]) + sh[99 + threadIdx.x];
}

// out[j] = sum_b part[b][j]: one workgroup per column j, each thread summing
// the rows t, t + 256, ... and the workgroup tree-summing those (fixed order)
__global__ void __launch_bounds__(256) k_colreduce(const float* __restrict__ part, int64_t nb,
                                                   int width, float* __restrict__ out) {
    __shared__ float sh[256];
    const int j = blockIdx.x;
    float s = 0.0f;
    for (int64_t b = threadIdx.x; b < nb; b += 256) s += part[b * width + j];
    s = block_sum256(s, sh);
    if (threadIdx.x == 0) out[j] = s;
}

__global__ void __launch_bounds__(256) k_sum(const float* __restrict__ a, int64_t n,
                                             float* __restrict__ part) {
    __shared__ float sh[256];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const float s = block_sum256(i < n ? a[i] : 0.0f, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// dy = 2 m (y - t) / msum; partial sums of m (y - t)^2
__global__ void __launch_bounds__(256) k_mse(const float* __restrict__ y, const float* __restrict__ t,
                                             const float* __restrict__ m, int64_t n,
                                             const float* __restrict__ msum,
                                             float* __restrict__ dy, float* __restrict__ part) {
    __shared__ float sh[256];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float l = 0.0f;
    if (i < n) {
        const float r = y[i] - t[i];
        const float mr = m[i] * r;
        dy[i] = 2.0f * mr / msum[0];
        l = mr * r;
    }
    const float s = block_sum256(l, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Adam (Kingma & Ba) with bias corrections c1 = 1 - b1^t, c2 = 1 - b2^t
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

// W[co][k] = master[co][k] (k < 27 cin) and Wt[ci][k'] with k' = (26 - off) cout + co
__global__ void k_pack(const float* __restrict__ master, int cin, int cout, int kp, int kpt,
                       bf16* __restrict__ W, bf16* __restrict__ Wt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nW = (int64_t)cout * kp, nT = (int64_t)cin * kpt;
    const int K = 27 * cin, Kt = 27 * cout;
    if (i < nW) {
        const int co = (int)(i / kp), k = (int)(i % kp);
        W[i] = (bf16)(k < K ? master[(int64_t)co * K + k] : 0.0f);
    } else if (Wt && i < nW + nT) {
        const int64_t j = i - nW;
        const int ci = (int)(j / kpt), kt = (int)(j % kpt);
        float val = 0.0f;
        if (kt < Kt) {
            const int offp = kt / cout, co = kt % cout;
            const int off = 26 - offp;
            val = master[((int64_t)co * 27 + off) * cin + ci];
        }
        Wt[j] = (bf16)val;
    }
}

// The weights in the brick convolution's order: for each block of 32 outputs
// cb, chunk of 32 inputs c, offset off and input group grp, the 32 outputs'
// eight channels in a row (16 bytes each), so that one dz plane of a chunk
// (9 offsets) is one contiguous run: element
//   ((((cb nch + c) 27 + off) 4 + grp) 32 + n) 8 + e
// holds output cb 32 + n, input c 32 + grp 8 + e (zero past the outputs).
// With `flip` the copy is of the data-gradient convolution: inputs are the
// layer's outputs, outputs its inputs, offsets mirrored.
__global__ void k_pack_w(const float* __restrict__ master, int cin, int cout, int flip,
                         bf16* __restrict__ wp) {
    const int ci_n = flip ? cout : cin, co_n = flip ? cin : cout;
    const int nch = ci_n / 32, ncb = (co_n + 31) / 32;
    const int64_t n_el = (int64_t)ncb * nch * 27 * 1024;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_el) return;
    const int e = (int)(i % 8), n = (int)((i / 8) % 32), grp = (int)((i / 256) % 4);
    const int off = (int)((i / 1024) % 27);
    const int64_t cc = i / (1024 * 27);
    const int c = (int)(cc % nch), cb = (int)(cc / nch);
    const int ci = c * 32 + grp * 8 + e, co = cb * 32 + n;
    float val = 0.0f;
    if (co < co_n)
        val = flip ? master[((int64_t)ci * 27 + (26 - off)) * cin + co]
                   : master[((int64_t)co * 27 + off) * cin + ci];
    wp[i] = (bf16)val;
}

// The first layer's copy (8 input channels) in k_conv_p8's order: element
//   (((cb 7 + s) 4 + kg) 32 + n) 8 + e
// holds output cb 32 + n, offset 4 s + kg (zero from 27 on), input e.
__global__ void k_pack_w8(const float* __restrict__ master, int cout, bf16* __restrict__ wp) {
    const int ncb = (cout + 31) / 32;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)ncb * 7 * 1024) return;
    const int e = (int)(i % 8), n = (int)((i / 8) % 32), kg = (int)((i / 256) % 4);
    const int st = (int)((i / 1024) % 7), cb = (int)(i / (1024 * 7));
    const int off = 4 * st + kg, co = cb * 32 + n;
    wp[i] = (bf16)(off < 27 && co < cout ? master[((int64_t)co * 27 + off) * 8 + e] : 0.0f);
}

int64_t packed_w_count(int cin_conv, int cout_conv) {
    if (cin_conv == 8) return (int64_t)((cout_conv + 31) / 32) * 7 * 1024;
    return (int64_t)((cout_conv + 31) / 32) * (cin_conv / 32) * 27 * 1024;
}

__device__ inline uint64_t mix64(uint64_t x) {
    x += 0x9e3779b97f4a7c15ULL;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ULL;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebULL;
    return x ^ (x >> 31);
}

// p[i] = std * N(0,1) by Box-Muller on two counter-based uniforms
__global__ void k_init_normal(float* __restrict__ p, int64_t n, float stdv, uint64_t seed,
                              uint64_t stream) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t a = mix64(seed ^ mix64(stream * 0x100000001b3ULL + 2 * (uint64_t)i));
    const uint64_t b = mix64(seed ^ mix64(stream * 0x100000001b3ULL + 2 * (uint64_t)i + 1));
    const double u1 = ((double)(a >> 11) + 1.0) / 9007199254740993.0;
    const double u2 = (double)(b >> 11) / 9007199254740992.0;
    p[i] = (float)(stdv * sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
}

__global__ void k_fill_f32(float* p, int64_t n, float v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_bf16_to_f32(const bf16* __restrict__ a, int ap, int ao, int C, int64_t V,
                              float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V * C) return;
    const int64_t v = i / C;
    const int c = (int)(i % C);
    out[i] = (float)a[v * ap + ao + c];
}

// ---------------------------------------------------------------------------
// Input rasterisation and FED-FEM resampling
// ---------------------------------------------------------------------------
// one sample of the network input (layout of fedsur_sample)
struct RasterSample {
    double cx, cy, cz, sigma, q0, k0, omega_b, ax, ay, az, hmesh, reserved;
};
struct RasterPhys {
    double rho0, c0, rhob_cb, t_heat;
};
static_assert(sizeof(RasterSample) == sizeof(fedsur_sample), "sample layout");

__device__ inline double cell_avg_1d(double x0, double h, double c, double s) {
    const double k = 1.0 / (s * 1.4142135623730951);
    return (s * 1.2533141373155003 / h) * (erf((x0 + h - c) * k) - erf((x0 - c) * k));
}

// Gauss-Legendre rule of order 8 on [-1, 1] (Abramowitz & Stegun, Table 25.4)
__constant__ double kGLx[4] = {0.1834346424956498, 0.5255324099163290, 0.7966664774136267,
                               0.9602898564975363};
__constant__ double kGLw[4] = {0.3626837833783620, 0.3137066458778873, 0.2223810344533745,
                               0.1012285362903763};

// Temperature rise at squared distance r2 from the centre of a Gaussian
// source switched on at t = 0 in an infinite medium of constant properties
// with perfusion: the heat released at time t - tau has spread to variance
// sigma^2 + 2 alpha tau and decayed by exp(-m tau), so
//   dT = Q0 / (rho c) int_0^t exp(-m tau) (s0 / s)^(3/2) exp(-r2 / (2 s)) dtau,
//   s = s0 + 2 alpha tau, s0 = sigma^2, alpha = k0 / (rho c),
//   m = omega_b rho_b c_b / (rho c).
// The integral is taken over the geometric pieces [0, t/128], [t/128, t/64],
// ..., [t/2, t] with 8 Gauss-Legendre points each (FP64).
__device__ double prior_rise(double r2, const RasterSample& p, const RasterPhys& ph) {
    const double rc = ph.rho0 * ph.c0;
    const double alpha = p.k0 / rc, m = p.omega_b * ph.rhob_cb / rc, s0 = p.sigma * p.sigma;
    double sum = 0.0, lo = 0.0, hi = ph.t_heat / 128.0;
    for (int seg = 0; seg < 8; seg++) {
        const double mid = 0.5 * (lo + hi), half = 0.5 * (hi - lo);
        for (int j = 0; j < 8; j++) {
            const double tau = mid + (j < 4 ? -half * kGLx[j] : half * kGLx[j - 4]);
            const double sv = s0 + 2.0 * alpha * tau;
            const double g = s0 / sv;
            sum += half * kGLw[j & 3] * exp(-m * tau - 0.5 * r2 / sv) * g * sqrt(g);
        }
        lo = hi;
        hi *= 2.0;
    }
    return p.q0 / rc * sum;
}

// Term j (piece j / 8, point j % 8) of the same quadrature, split into what
// depends on the sample only: the term is c exp(-a r2) with
//   c = Q0 / (rho c) (half w) exp(-m tau) g^(3/2),  a = 1 / (2 s).
__device__ void prior_term(int j, const RasterSample& p, const RasterPhys& ph, double& c,
                           double& a) {
    const double rc = ph.rho0 * ph.c0;
    const double alpha = p.k0 / rc, m = p.omega_b * ph.rhob_cb / rc, s0 = p.sigma * p.sigma;
    const int seg = j >> 3, k = j & 7;
    const double hi = ph.t_heat / 128.0 * (double)(1 << seg), lo = seg == 0 ? 0.0 : 0.5 * hi;
    const double mid = 0.5 * (lo + hi), half = 0.5 * (hi - lo);
    const double tau = mid + (k < 4 ? -half * kGLx[k] : half * kGLx[k - 4]);
    const double sv = s0 + 2.0 * alpha * tau;
    const double g = s0 / sv;
    c = p.q0 / rc * half * kGLw[k & 3] * exp(-m * tau) * g * sqrt(g);
    a = 0.5 / sv;
}

__global__ void k_prior_scale(int B, const RasterSample* __restrict__ smp, RasterPhys ph,
                              float* __restrict__ scale) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < B) scale[b] = (float)prior_rise(0.0, smp[b], ph);
}

__global__ void __launch_bounds__(256) k_rasterize(int G, double fx, double fy, double fz,
                                                    double h, int B,
                                                    const RasterSample* __restrict__ smp,
                                                    RasterPhys ph,
                                                    const float* __restrict__ scale,
                                                    bf16* __restrict__ x,
                                                    float* __restrict__ prior) {
    // the prior's 64 quadrature terms of the block's first sample, once per
    // block; a voxel of another sample (a block straddling two) takes the
    // quadrature directly
    __shared__ double tc[64], ta[64];
    const int64_t G3 = (int64_t)G * G * G;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x;
    const int64_t b0 = i0 / G3;
    if (threadIdx.x < 64) prior_term(threadIdx.x, smp[b0], ph, tc[threadIdx.x], ta[threadIdx.x]);
    __syncthreads();
    const int64_t i = i0 + threadIdx.x;
    if (i >= (int64_t)B * G3) return;
    const int64_t b = i / G3;
    const int64_t r = i - b * G3;
    const int iz = (int)(r / ((int64_t)G * G)), iy = (int)((r / G) % G), ix = (int)(r % G);
    const RasterSample p = smp[b];
    // voxel average of the source shape exp(-|x - c|^2 / (2 sigma^2))
    const double q = cell_avg_1d(fx + ix * h, h, p.cx, p.sigma) *
                     cell_avg_1d(fy + iy * h, h, p.cy, p.sigma) *
                     cell_avg_1d(fz + iz * h, h, p.cz, p.sigma);
    // voxel centre, relative to the source and to the frame centre
    const double half = 0.5 * G * h;
    const double vx = fx + (ix + 0.5) * h, vy = fy + (iy + 0.5) * h, vz = fz + (iz + 0.5) * h;
    const double ex = (vx - fx - half) / p.ax, ey = (vy - fy - half) / p.ay,
                 ez = (vz - fz - half) / p.az;
    const float mk = (ex * ex + ey * ey + ez * ez <= 1.0) ? 1.0f : 0.0f;
    const double r2 = (vx - p.cx) * (vx - p.cx) + (vy - p.cy) * (vy - p.cy) + (vz - p.cz) * (vz - p.cz);
    double pr;
    if (b == b0) {
        // FP32 exponentials: a term's error stays below 1e-7 of its c (the
        // argument x = a r2 rounded to FP32 moves it by at most x e^-x 2^-24,
        // expf adds its own ulp), and the terms are summed in FP64
        pr = 0.0;
#pragma unroll 8
        for (int j = 0; j < 64; j++) pr += tc[j] * (double)expf((float)(-ta[j] * r2));
    } else {
        pr = prior_rise(r2, p, ph);
    }
    const float P = scale[b];
    bf16x8 o;
    o[0] = (bf16)(float)q;
    o[1] = (bf16)(mk * (float)((p.k0 - 0.525) / 0.075));
    o[2] = (bf16)(mk * (float)((p.omega_b - 0.011) / 0.009));
    o[3] = (bf16)mk;
    o[4] = (bf16)(float)(pr / P);
    o[5] = (bf16)(mk * (float)(pr * 0.01));
    o[6] = (bf16)(mk * (float)(p.hmesh / 2e-3 - 1.0));
    o[7] = (bf16)(mk * (float)(p.sigma / 4e-3 - 1.0));
    *reinterpret_cast<bf16x8*>(x + i * 8) = o;
    if (prior) prior[i] = (float)pr;
}

// target = (T - Ta - prior) / P inside the mesh (0 outside); loss weight
// 1 + focus prior / P inside the mesh, 0 outside
__global__ void k_target(int64_t G3, int B, const float* __restrict__ prior,
                         const float* __restrict__ scale, const float* __restrict__ T,
                         const uint8_t* __restrict__ mask, float Ta, float focus,
                         float* __restrict__ target, float* __restrict__ weight) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * G3) return;
    const float P = scale[i / G3];
    const bool in = mask[i] != 0;
    target[i] = in ? (T[i] - Ta - prior[i]) / P : 0.0f;
    weight[i] = in ? 1.0f + focus * fmaxf(prior[i] / P, 0.0f) : 0.0f;
}

// y <- Ta + prior + P y (the predicted temperature)
__global__ void k_decode(int64_t G3, int B, const float* __restrict__ prior,
                         const float* __restrict__ scale, float Ta, float* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * G3) return;
    y[i] = Ta + (prior[i] + scale[i / G3] * y[i]);
}

// err[b] = max over the mesh's voxels of |Tp - T|; non-negative floats
// order like their bit patterns, so the maximum is an integer atomic max
// (NaN, whose pattern exceeds every finite one, propagates)
__global__ void __launch_bounds__(256) k_max_err(int64_t G3, int B, const float* __restrict__ Tp,
                                                 const float* __restrict__ T,
                                                 const uint8_t* __restrict__ mask,
                                                 unsigned* __restrict__ err) {
    __shared__ unsigned sh[256];
    const int b = blockIdx.y;
    unsigned m = 0u;
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < G3; v += (int64_t)gridDim.x * 256) {
        const int64_t i = (int64_t)b * G3 + v;
        if (mask[i]) {
            const float d = fabsf(Tp[i] - T[i]);
            m = max(m, __float_as_uint(d));
        }
    }
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] = max(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(err + b, sh[0]);
}

__global__ void k_fill_u32(unsigned* p, int n, unsigned v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

struct ResampleArgs {
    int64_t E;
    const double* xyz;
    const int32_t* conn;
    const void* T;
    int fp32c;
    int G;
    double fx, fy, fz, h;
    int32_t* owner;
    float* out;
    uint8_t* mask;
};

// barycentric coordinates of p in tet e (returns false if degenerate)
__device__ bool bary(const ResampleArgs& a, int64_t e, const double* p, double lam[4]) {
    double q[4][3];
    for (int c = 0; c < 4; c++) {
        const int64_t n = a.conn[4 * e + c];
        for (int d = 0; d < 3; d++) q[c][d] = a.xyz[3 * n + d];
    }
    double e1[3], e2[3], e3[3], r[3];
    for (int d = 0; d < 3; d++) {
        e1[d] = q[1][d] - q[0][d];
        e2[d] = q[2][d] - q[0][d];
        e3[d] = q[3][d] - q[0][d];
        r[d] = p[d] - q[0][d];
    }
    const double c23[3] = {e2[1] * e3[2] - e2[2] * e3[1], e2[2] * e3[0] - e2[0] * e3[2],
                           e2[0] * e3[1] - e2[1] * e3[0]};
    const double c31[3] = {e3[1] * e1[2] - e3[2] * e1[1], e3[2] * e1[0] - e3[0] * e1[2],
                           e3[0] * e1[1] - e3[1] * e1[0]};
    const double c12[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                           e1[0] * e2[1] - e1[1] * e2[0]};
    const double det = e1[0] * c23[0] + e1[1] * c23[1] + e1[2] * c23[2];
    if (det == 0.0) return false;
    lam[1] = (r[0] * c23[0] + r[1] * c23[1] + r[2] * c23[2]) / det;
    lam[2] = (r[0] * c31[0] + r[1] * c31[1] + r[2] * c31[2]) / det;
    lam[3] = (r[0] * c12[0] + r[1] * c12[1] + r[2] * c12[2]) / det;
    lam[0] = 1.0 - lam[1] - lam[2] - lam[3];
    return true;
}

template <int PASS>
__global__ void k_resample(ResampleArgs a) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.E) return;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int c = 0; c < 4; c++) {
        const int64_t n = a.conn[4 * e + c];
        for (int d = 0; d < 3; d++) {
            lo[d] = fmin(lo[d], a.xyz[3 * n + d]);
            hi[d] = fmax(hi[d], a.xyz[3 * n + d]);
        }
    }
    const double f[3] = {a.fx, a.fy, a.fz};
    int i0[3], i1[3];
    for (int d = 0; d < 3; d++) {
        i0[d] = max(0, (int)ceil((lo[d] - f[d]) / a.h - 0.5));
        i1[d] = min(a.G - 1, (int)floor((hi[d] - f[d]) / a.h - 0.5));
    }
    for (int iz = i0[2]; iz <= i1[2]; iz++)
        for (int iy = i0[1]; iy <= i1[1]; iy++)
            for (int ix = i0[0]; ix <= i1[0]; ix++) {
                const double p[3] = {f[0] + (ix + 0.5) * a.h, f[1] + (iy + 0.5) * a.h,
                                     f[2] + (iz + 0.5) * a.h};
                double lam[4];
                if (!bary(a, e, p, lam)) continue;
                if (lam[0] < -1e-10 || lam[1] < -1e-10 || lam[2] < -1e-10 || lam[3] < -1e-10)
                    continue;
                const int64_t v = ((int64_t)iz * a.G + iy) * a.G + ix;
                if (PASS == 0) {
                    atomicMin(&a.owner[v], (int32_t)e);
                } else if (a.owner[v] == (int32_t)e) {
                    double T = 0.0;
                    for (int c = 0; c < 4; c++) {
                        const int64_t n = a.conn[4 * e + c];
                        double Tn;
                        if (a.fp32c) {
                            const float2 s = static_cast<const float2*>(a.T)[n];
                            Tn = (double)s.x + (double)s.y;
                        } else {
                            Tn = static_cast<const double*>(a.T)[n];
                        }
                        T += lam[c] * Tn;
                    }
                    a.out[v] = (float)T;
                    a.mask[v] = 1;
                }
            }
}

__global__ void k_resample_clear(int64_t n, int32_t* owner, float* out, uint8_t* mask) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    owner[i] = INT32_MAX;
    out[i] = 0.0f;
    mask[i] = 0;
}

// ---------------------------------------------------------------------------
// Network description
// ---------------------------------------------------------------------------
struct LayerDef {
    int cin, cout, lvl;
};
const LayerDef kLayers[FEDSUR_LAYERS] = {{8, 32, 0},    {32, 32, 0},  {32, 64, 1},  {64, 64, 1},
                                         {64, 128, 2},  {128, 128, 2}, {192, 64, 1}, {64, 64, 1},
                                         {96, 32, 0},   {32, 32, 0}};
enum { E1A, E1B, E2A, E2B, E3A, E3B, D2A, D2B, D1A, D1B };

struct View {
    bf16* p;
    int pitch, off, c, lvl;
};

}  // namespace

struct fedsur_net {
    int G = 0, Bmax = 0, device = 0;
    hipStream_t own = nullptr, stream = nullptr;
    int64_t nparams = 0;
    int64_t w_off[FEDSUR_LAYERS], b_off[FEDSUR_LAYERS], head_off = 0;
    int kp[FEDSUR_LAYERS], kpt[FEDSUR_LAYERS], kp2[FEDSUR_LAYERS];
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;  // FP32 master etc.
    bf16 *W[FEDSUR_LAYERS], *Wt[FEDSUR_LAYERS];
    // brick-order copies for the brick convolutions (null if the layer's
    // input, resp. output, channels are neither 8 nor a multiple of 32, resp.
    // not a multiple of 32)
    bf16 *Wp[FEDSUR_LAYERS], *Wtp[FEDSUR_LAYERS];
    // activations
    bf16 *e1a, *cat1, *p1, *e2a, *cat2, *p2, *e3a, *e3b, *d2a, *d2b, *d1a, *d1b;
    float* y = nullptr;
    // gradients
    float *dy = nullptr, *red = nullptr, *part = nullptr, *scal = nullptr;
    int64_t part_cap = 0, red_cap = 0;
    bf16 *gA0, *gB0, *gcat1, *gA1, *gB1, *gcat2, *gA2, *gB2, *gp1, *gp2;
    int64_t adam_t = 0;
    std::vector<void*> allocs;
    int B = 0;  // batch of the last forward
};

namespace {

int64_t vox(const fedsur_net* n, int lvl, int B) {
    const int64_t g = n->G >> lvl;
    return (int64_t)B * g * g * g;
}

template <typename T>
hipError_t nalloc(fedsur_net* n, T** p, size_t count) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(16, count * sizeof(T)));
    if (e != hipSuccess) return e;
    n->allocs.push_back(q);
    *p = static_cast<T*>(q);
    return hipSuccess;
}

View out_view(fedsur_net* n, int L) {
    switch (L) {
        case E1A: return {n->e1a, 32, 0, 32, 0};
        case E1B: return {n->cat1, 96, 64, 32, 0};
        case E2A: return {n->e2a, 64, 0, 64, 1};
        case E2B: return {n->cat2, 192, 128, 64, 1};
        case E3A: return {n->e3a, 128, 0, 128, 2};
        case E3B: return {n->e3b, 128, 0, 128, 2};
        case D2A: return {n->d2a, 64, 0, 64, 1};
        case D2B: return {n->d2b, 64, 0, 64, 1};
        case D1A: return {n->d1a, 32, 0, 32, 0};
        default: return {n->d1b, 32, 0, 32, 0};
    }
}

View in_view(fedsur_net* n, int L, const bf16* x) {
    switch (L) {
        case E1A: return {const_cast<bf16*>(x), 8, 0, 8, 0};
        case E1B: return {n->e1a, 32, 0, 32, 0};
        case E2A: return {n->p1, 32, 0, 32, 1};
        case E2B: return {n->e2a, 64, 0, 64, 1};
        case E3A: return {n->p2, 64, 0, 64, 2};
        case E3B: return {n->e3a, 128, 0, 128, 2};
        case D2A: return {n->cat2, 192, 0, 192, 1};
        case D2B: return {n->d2a, 64, 0, 64, 1};
        case D1A: return {n->cat1, 96, 0, 96, 0};
        default: return {n->d1a, 32, 0, 32, 0};
    }
}

// D2A's and D1A's leading input channels are the upsampled output of the
// level below (e3b: 128, d2b: 64).  On grids of 16k the brick kernels read
// them at the parent voxel instead of from a written copy in cat2 / cat1.
struct UpSrc {
    const bf16* p;
    int pitch, c;
};
UpSrc up_source(const fedsur_net* n, int L) {
    const int G = n->G >> kLayers[L].lvl;
    if (G % 16) return {nullptr, 0, 0};
    if (L == D2A) return {n->e3b, 128, 128};
    if (L == D1A) return {n->d2b, 64, 64};
    return {nullptr, 0, 0};
}

// E1B's and E2B's outputs are pooled for the level below (p1: 32, p2: 64
// channels); on grids of 16k the brick kernel writes the means itself.
bf16* pool_target(const fedsur_net* n, int L, int& pitch) {
    const int G = n->G >> kLayers[L].lvl;
    pitch = 0;
    if (G % 16) return nullptr;
    if (L == E1B) return pitch = 32, n->p1;
    if (L == E2B) return pitch = 64, n->p2;
    return nullptr;
}

hipError_t run_conv(fedsur_net* n, int L, const bf16* x, int B) {
    const View in = in_view(n, L, x), out = out_view(n, L);
    ConvArgs a;
    a.in = in.p;
    a.ip = in.pitch;
    a.io = in.off;
    a.cin = kLayers[L].cin;
    a.w = n->W[L];
    a.kp = n->kp[L];
    a.wp = reinterpret_cast<const uint4*>(n->Wp[L]);
    const UpSrc u = up_source(n, L);
    a.up = u.p;
    a.upp = u.pitch;
    a.upo = 0;
    a.upc = u.c;
    a.pool = pool_target(n, L, a.pp);
    a.bias = n->p + n->b_off[L];
    a.out = out.p;
    a.op = out.pitch;
    a.oo = out.off;
    a.cout = kLayers[L].cout;
    a.G = n->G >> kLayers[L].lvl;
    a.ks = 3;
    a.relu = 1;
    a.V = vox(n, kLayers[L].lvl, B);
    return conv_fwd(a, n->stream);
}

// weight/bias gradients of layer L from its pre-activation gradient dpre
// (contiguous [V][cout], the producer having applied L's ReLU), then (if dx)
// the gradient of its input into dx, passed through the ReLU whose output is
// dxmask when one is given (the layer below): fused into the brick kernel's
// epilogue, or an in-place pass after the gathered kernels
hipError_t conv_backward(fedsur_net* n, int L, const bf16* x, int B, const bf16* dpre,
                         const View* dx, const View* dxmask) {
    const LayerDef& d = kLayers[L];
    const View in = in_view(n, L, x);
    const int64_t V = vox(n, d.lvl, B);
    const int G = n->G >> d.lvl;
    hipStream_t s = n->stream;
    // weight and bias gradient: ~kWgradBlocks (brick form: kWgradBrickBlocks)
    // workgroups over tiles x splits
    const bool brick = G % 16 == 0 && d.cin % 32 == 0 && d.cout % 32 == 0;
    const int KN = wgrad_kn(d.cout), COT = wgrad_cot(d.cout);
    const int kb = brick ? d.cin / 32 : n->kp2[L] / KN;
    const int cb = brick ? d.cout / 32 : (d.cout + COT - 1) / COT;
    int64_t splits = 0, per = 0, vsplit = 0;
    if (brick) {
        // runs of whole bricks; the partial buffer bounds the number of runs
        const int64_t nbr = V / 256;
        // at most one workgroup per CU in all (a second round would run alone)
        const int64_t want = std::max<int64_t>(1, kWgradBrickBlocks / (kb * cb));
        const int64_t cap = n->part_cap / ((int64_t)d.cout * n->kp2[L]);
        splits = std::max<int64_t>(1, std::min({want, nbr, cap, (int64_t)65535}));
        per = (nbr + splits - 1) / splits;
        splits = (nbr + per - 1) / per;
    } else {
        vsplit = wgrad_vsplit(V, kb * cb);
        splits = (V + vsplit - 1) / vsplit;
    }
    if (splits * d.cout * n->kp2[L] > n->part_cap || splits > 65535) return hipErrorInvalidValue;
    WgradArgs w;
    w.d = dpre;
    w.dp = d.cout;
    w.doff = 0;
    w.cout = d.cout;
    w.in = in.p;
    w.ip = in.pitch;
    w.io = in.off;
    w.cin = d.cin;
    const UpSrc u = up_source(n, L);
    if (u.c && !brick) return hipErrorInvalidValue;
    w.up = u.p;
    w.upp = u.pitch;
    w.upo = 0;
    w.upc = u.c;
    w.G = G;
    w.V = V;
    w.vsplit = vsplit;
    w.kp2 = n->kp2[L];
    w.part = n->part;
    if (brick) {
        hipLaunchKernelGGL(k_wgrad_brick<32>, dim3((unsigned)kb, (unsigned)cb, (unsigned)splits),
                           dim3(512), 0, s, w, per);
        if (hipError_t e0 = hipGetLastError()) return e0;
    } else if (hipError_t e0 = launch_wgrad(w, kb, cb, splits, s)) {
        return e0;
    }
    const int64_t nred = (int64_t)d.cout * 27 * d.cin + d.cout;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(nblocks(nred, 64)), dim3(256), 0, s, n->part,
                       (int)splits, d.cout, n->kp2[L], 27 * d.cin, n->g + n->w_off[L],
                       n->g + n->b_off[L]);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !dx) return e;
    ConvArgs a;
    a.in = dpre;
    a.ip = d.cout;
    a.io = 0;
    a.cin = d.cout;
    a.w = n->Wt[L];
    a.kp = n->kpt[L];
    a.wp = reinterpret_cast<const uint4*>(n->Wtp[L]);
    a.bias = nullptr;
    a.out = dx->p;
    a.op = dx->pitch;
    a.oo = dx->off;
    a.cout = d.cin;
    a.G = G;
    a.ks = 3;
    a.relu = 0;
    a.V = V;
    const bool fuse_mask = dxmask && G % 16 == 0 && d.cout % 32 == 0 && a.wp;
    if (fuse_mask) {
        a.mk = dxmask->p;
        a.mkp = dxmask->pitch;
        a.mko = dxmask->off;
    }
    if (hipError_t e1 = conv_fwd(a, s)) return e1;
    if (dxmask && !fuse_mask) {
        if (dx->pitch != d.cin || dx->off) return hipErrorInvalidValue;
        // dx is contiguous here ([V][cin]); each element is read, then written
        hipLaunchKernelGGL(k_relu_bwd, dim3(nblocks(V * (d.cin / 8), 256)), dim3(256), 0, s,
                           dx->p, dx->pitch, dx->off, dxmask->p, dxmask->pitch, dxmask->off,
                           d.cin, V, dx->p);
    }
    return hipGetLastError();
}

hipError_t pack_all(fedsur_net* n) {
    for (int L = 0; L < FEDSUR_LAYERS; L++) {
        const LayerDef& d = kLayers[L];
        const int64_t tot = (int64_t)d.cout * n->kp[L] + (int64_t)d.cin * n->kpt[L];
        hipLaunchKernelGGL(k_pack, dim3(nblocks(tot, 256)), dim3(256), 0, n->stream,
                           n->p + n->w_off[L], d.cin, d.cout, n->kp[L], n->kpt[L], n->W[L],
                           n->Wt[L]);
        if (n->Wp[L] && d.cin == 8)
            hipLaunchKernelGGL(k_pack_w8, dim3(nblocks(packed_w_count(d.cin, d.cout), 256)),
                               dim3(256), 0, n->stream, n->p + n->w_off[L], d.cout, n->Wp[L]);
        else if (n->Wp[L])
            hipLaunchKernelGGL(k_pack_w, dim3(nblocks(packed_w_count(d.cin, d.cout), 256)),
                               dim3(256), 0, n->stream, n->p + n->w_off[L], d.cin, d.cout, 0,
                               n->Wp[L]);
        if (n->Wtp[L])
            hipLaunchKernelGGL(k_pack_w, dim3(nblocks(packed_w_count(d.cout, d.cin), 256)),
                               dim3(256), 0, n->stream, n->p + n->w_off[L], d.cin, d.cout, 1,
                               n->Wtp[L]);
    }
    return hipGetLastError();
}

hipError_t reduce_to(fedsur_net* n, const float* a, int64_t len, float* out) {
    // two fixed-order passes: block sums, then one block over the partials
    const int64_t nb = (len + 255) / 256;
    if (nb > n->red_cap) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sum, dim3((unsigned)nb), dim3(256), 0, n->stream, a, len, n->red);
    hipLaunchKernelGGL(k_colreduce, dim3(1), dim3(256), 0, n->stream, n->red, nb, 1, out);
    return hipGetLastError();
}

hipError_t forward_impl(fedsur_net* n, int B, const bf16* x, float* y) {
    hipStream_t s = n->stream;
    const int G = n->G;
    hipError_t e;
    if ((e = run_conv(n, E1A, x, B)) || (e = run_conv(n, E1B, x, B))) return e;
    int pp;
    if (!pool_target(n, E1B, pp))
        hipLaunchKernelGGL(k_pool_fwd, dim3(nblocks(vox(n, 1, B) * 4, 256)), dim3(256), 0, s,
                           n->cat1, 96, 64, 32, G, B, n->p1);
    if ((e = run_conv(n, E2A, x, B)) || (e = run_conv(n, E2B, x, B))) return e;
    if (!pool_target(n, E2B, pp))
        hipLaunchKernelGGL(k_pool_fwd, dim3(nblocks(vox(n, 2, B) * 8, 256)), dim3(256), 0, s,
                           n->cat2, 192, 128, 64, G / 2, B, n->p2);
    if ((e = run_conv(n, E3A, x, B)) || (e = run_conv(n, E3B, x, B))) return e;
    if (!up_source(n, D2A).c)
        hipLaunchKernelGGL(k_up_fwd, dim3(nblocks(vox(n, 2, B) * 16, 256)), dim3(256), 0, s,
                           n->e3b, 128, G / 2, B, n->cat2, 192, 0);
    if ((e = run_conv(n, D2A, x, B)) || (e = run_conv(n, D2B, x, B))) return e;
    if (!up_source(n, D1A).c)
        hipLaunchKernelGGL(k_up_fwd, dim3(nblocks(vox(n, 1, B) * 8, 256)), dim3(256), 0, s,
                           n->d2b, 64, G, B, n->cat1, 96, 0);
    if ((e = run_conv(n, D1A, x, B)) || (e = run_conv(n, D1B, x, B))) return e;
    hipLaunchKernelGGL(k_head_fwd, dim3(nblocks(vox(n, 0, B), 256)), dim3(256), 0, s, n->d1b,
                       n->p + n->head_off, vox(n, 0, B), y);
    n->B = B;
    return hipGetLastError();
}

hipError_t backward_impl(fedsur_net* n, int B, const bf16* x) {
    hipStream_t s = n->stream;
    const int G = n->G;
    const int64_t V0 = vox(n, 0, B), V1 = vox(n, 1, B), V2 = vox(n, 2, B);
    hipError_t e;
    // Every gradient handed to conv_backward is pre-activation: its producer
    // (the head, a 2 x 2 x 2 pass or the layer above's data gradient) applies
    // the layer's ReLU.  Pre-activation gradients alternate between the gA*
    // and gB* buffers of each level.
    // head: dL/d(d1b) through d1b's ReLU into gA0 [V0][32], head partials
    const int64_t nb = (V0 + 255) / 256;
    if (nb * 33 > n->part_cap) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_head_bwd, dim3((unsigned)nb), dim3(256), 0, s, n->dy, n->d1b,
                       n->p + n->head_off, V0, n->gA0, n->part);
    hipLaunchKernelGGL(k_colreduce, dim3(33), dim3(256), 0, s, n->part, nb, 33, n->g + n->head_off);
    const View gB0{n->gB0, 32, 0, 32, 0}, gB1{n->gB1, 64, 0, 64, 1};
    const View gB2{n->gB2, 128, 0, 128, 2};
    const View gc1{n->gcat1, 96, 0, 96, 0}, gc2{n->gcat2, 192, 0, 192, 1};
    const View gp1{n->gp1, 32, 0, 32, 1}, gp2{n->gp2, 64, 0, 64, 2};
    const View o_d1a = out_view(n, D1A), o_d2a = out_view(n, D2A), o_e3a = out_view(n, E3A);
    const View o_e2a = out_view(n, E2A), o_e1a = out_view(n, E1A);
    const View o_d2b = out_view(n, D2B), o_e3b = out_view(n, E3B);
    const View o_e2b = out_view(n, E2B), o_e1b = out_view(n, E1B);
    // d1b (input d1a, through d1a's ReLU -> gB0), d1a (input cat1 -> gcat1)
    if ((e = conv_backward(n, D1B, x, B, n->gA0, &gB0, &o_d1a))) return e;
    if ((e = conv_backward(n, D1A, x, B, n->gB0, &gc1, nullptr))) return e;
    // upsample backward: channels [0, 64) of gcat1, through d2b's ReLU -> gA1
    hipLaunchKernelGGL(k_up_bwd, dim3(nblocks(V1 * 8, 256)), dim3(256), 0, s, n->gcat1, 96, 0, 64,
                       G, B, o_d2b.p, o_d2b.pitch, o_d2b.off, n->gA1);
    if ((e = conv_backward(n, D2B, x, B, n->gA1, &gB1, &o_d2a))) return e;
    if ((e = conv_backward(n, D2A, x, B, n->gB1, &gc2, nullptr))) return e;
    // channels [0, 128) of gcat2, through e3b's ReLU -> gA2 [V2][128]
    hipLaunchKernelGGL(k_up_bwd, dim3(nblocks(V2 * 16, 256)), dim3(256), 0, s, n->gcat2, 192, 0,
                       128, G / 2, B, o_e3b.p, o_e3b.pitch, o_e3b.off, n->gA2);
    if ((e = conv_backward(n, E3B, x, B, n->gA2, &gB2, &o_e3a))) return e;
    if ((e = conv_backward(n, E3A, x, B, n->gB2, &gp2, nullptr))) return e;
    // g(e2b) = gcat2[:, 128:192] + pool backward of g(p2), through e2b's ReLU
    // -> gA1
    hipLaunchKernelGGL(k_pool_bwd_add, dim3(nblocks(V2 * 8, 256)), dim3(256), 0, s, n->gcat2, 192,
                       128, n->gp2, 64, G / 2, B, o_e2b.p, o_e2b.pitch, o_e2b.off, n->gA1);
    if ((e = conv_backward(n, E2B, x, B, n->gA1, &gB1, &o_e2a))) return e;
    if ((e = conv_backward(n, E2A, x, B, n->gB1, &gp1, nullptr))) return e;
    // g(e1b) = gcat1[:, 64:96] + pool backward of g(p1), through e1b's ReLU
    // -> gA0
    hipLaunchKernelGGL(k_pool_bwd_add, dim3(nblocks(V1 * 4, 256)), dim3(256), 0, s, n->gcat1, 96,
                       64, n->gp1, 32, G, B, o_e1b.p, o_e1b.pitch, o_e1b.off, n->gA0);
    if ((e = conv_backward(n, E1B, x, B, n->gA0, &gB0, &o_e1a))) return e;
    if ((e = conv_backward(n, E1A, x, B, n->gB0, nullptr, nullptr))) return e;
    return hipGetLastError();
}

void destroy_net(fedsur_net* n) {
    if (!n) return;
    (void)hipSetDevice(n->device);
    if (n->own) (void)hipStreamSynchronize(n->own);
    for (void* p : n->allocs) (void)hipFree(p);
    if (n->own) (void)hipStreamDestroy(n->own);
    delete n;
}

#define NCHK(expr)                                       \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return FEDFEM_E_HIP;       \
    } while (0)

}  // namespace

extern "C" {

int fedsur_create(int32_t grid, int32_t batch_max, uint64_t seed, fedsur_net** out) {
    if (!out || grid < 4 || grid % 4 || grid > 256 || batch_max < 1 || batch_max > 4096 ||
        (int64_t)batch_max * grid * grid * grid >= (int64_t(1) << 31))
        return FEDFEM_E_INVALID;
    *out = nullptr;
    fedsur_net* n = new (std::nothrow) fedsur_net();
    if (!n) return FEDFEM_E_NOMEM;
    n->G = grid;
    n->Bmax = batch_max;
    auto fail = [&](int code) {
        destroy_net(n);
        return code;
    };
    if (hipGetDevice(&n->device) != hipSuccess) return fail(FEDFEM_E_HIP);
    // a blocking stream: ordered with work on the legacy default stream, where
    // callers (and torch's default stream) put the inputs the network reads
    if (hipStreamCreateWithFlags(&n->own, hipStreamDefault) != hipSuccess)
        return fail(FEDFEM_E_HIP);
    n->stream = n->own;
    int64_t off = 0;
    int64_t max_part = 0;
    for (int L = 0; L < FEDSUR_LAYERS; L++) {
        const LayerDef& d = kLayers[L];
        n->w_off[L] = off;
        off += (int64_t)d.cout * 27 * d.cin;
        n->b_off[L] = off;
        off += d.cout;
        n->kp[L] = round_up(27 * d.cin, 32);
        n->kpt[L] = round_up(27 * d.cout, 32);
        // room for the bias column k = 27 cin; whole KN tiles
        n->kp2[L] = round_up(27 * d.cin + 1, wgrad_kn(d.cout));
        const int tiles = (n->kp2[L] / wgrad_kn(d.cout)) *
                          ((d.cout + wgrad_cot(d.cout) - 1) / wgrad_cot(d.cout));
        const int64_t max_splits = std::max(1, (kWgradBlocks + tiles - 1) / tiles);
        max_part = std::max(max_part, max_splits * d.cout * n->kp2[L]);
    }
    n->head_off = off;
    off += 33;
    n->nparams = off;
    const int B = batch_max;
    const int64_t V0 = vox(n, 0, B), V1 = vox(n, 1, B), V2 = vox(n, 2, B);
    bool ok = nalloc(n, &n->p, off) == hipSuccess && nalloc(n, &n->g, off) == hipSuccess &&
              nalloc(n, &n->m, off) == hipSuccess && nalloc(n, &n->v, off) == hipSuccess;
    for (int L = 0; ok && L < FEDSUR_LAYERS; L++) {
        const LayerDef& d = kLayers[L];
        ok = nalloc(n, &n->W[L], (size_t)d.cout * n->kp[L]) == hipSuccess &&
             nalloc(n, &n->Wt[L], (size_t)d.cin * n->kpt[L]) == hipSuccess;
        n->Wp[L] = n->Wtp[L] = nullptr;
        if (ok && (d.cin % 32 == 0 || d.cin == 8))
            ok = nalloc(n, &n->Wp[L], (size_t)packed_w_count(d.cin, d.cout)) == hipSuccess;
        if (ok && d.cout % 32 == 0)
            ok = nalloc(n, &n->Wtp[L], (size_t)packed_w_count(d.cout, d.cin)) == hipSuccess;
    }
    ok = ok && nalloc(n, &n->e1a, V0 * 32) == hipSuccess &&
         nalloc(n, &n->cat1, V0 * 96) == hipSuccess && nalloc(n, &n->p1, V1 * 32) == hipSuccess &&
         nalloc(n, &n->e2a, V1 * 64) == hipSuccess && nalloc(n, &n->cat2, V1 * 192) == hipSuccess &&
         nalloc(n, &n->p2, V2 * 64) == hipSuccess && nalloc(n, &n->e3a, V2 * 128) == hipSuccess &&
         nalloc(n, &n->e3b, V2 * 128) == hipSuccess && nalloc(n, &n->d2a, V1 * 64) == hipSuccess &&
         nalloc(n, &n->d2b, V1 * 64) == hipSuccess && nalloc(n, &n->d1a, V0 * 32) == hipSuccess &&
         nalloc(n, &n->d1b, V0 * 32) == hipSuccess && nalloc(n, &n->y, V0) == hipSuccess &&
         nalloc(n, &n->dy, V0) == hipSuccess && nalloc(n, &n->gA0, V0 * 32) == hipSuccess &&
         nalloc(n, &n->gB0, V0 * 32) == hipSuccess && nalloc(n, &n->gcat1, V0 * 96) == hipSuccess &&
         nalloc(n, &n->gA1, V1 * 64) == hipSuccess && nalloc(n, &n->gB1, V1 * 64) == hipSuccess &&
         nalloc(n, &n->gcat2, V1 * 192) == hipSuccess && nalloc(n, &n->gA2, V2 * 128) == hipSuccess &&
         nalloc(n, &n->gB2, V2 * 128) == hipSuccess && nalloc(n, &n->gp1, V1 * 32) == hipSuccess &&
         nalloc(n, &n->gp2, V2 * 64) == hipSuccess && nalloc(n, &n->scal, 8) == hipSuccess;
    // split-K partials: at most 128 voxel splits per layer; head partials too
    n->part_cap = std::max<int64_t>(max_part, ((V0 + 255) / 256) * 33);
    n->red_cap = (V0 + 255) / 256 + 1;
    ok = ok && nalloc(n, &n->part, n->part_cap) == hipSuccess &&
         nalloc(n, &n->red, n->red_cap) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        return fail(FEDFEM_E_NOMEM);
    }
    // He initialisation, zero biases and moments
    hipStream_t s = n->stream;
    for (int L = 0; L < FEDSUR_LAYERS; L++) {
        const LayerDef& d = kLayers[L];
        const int64_t cnt = (int64_t)d.cout * 27 * d.cin;
        hipLaunchKernelGGL(k_init_normal, dim3(nblocks(cnt, 256)), dim3(256), 0, s,
                           n->p + n->w_off[L], cnt, (float)std::sqrt(2.0 / (27.0 * d.cin)), seed,
                           (uint64_t)L);
        hipLaunchKernelGGL(k_fill_f32, dim3(1), dim3(128), 0, s, n->p + n->b_off[L],
                           (int64_t)d.cout, 0.0f);
    }
    hipLaunchKernelGGL(k_init_normal, dim3(1), dim3(64), 0, s, n->p + n->head_off, (int64_t)32,
                       (float)std::sqrt(1.0 / 32.0), seed, (uint64_t)FEDSUR_LAYERS);
    hipLaunchKernelGGL(k_fill_f32, dim3(1), dim3(1), 0, s, n->p + n->head_off + 32, (int64_t)1,
                       0.0f);
    hipLaunchKernelGGL(k_fill_f32, dim3(nblocks(off, 256)), dim3(256), 0, s, n->m, off, 0.0f);
    hipLaunchKernelGGL(k_fill_f32, dim3(nblocks(off, 256)), dim3(256), 0, s, n->v, off, 0.0f);
    hipLaunchKernelGGL(k_fill_f32, dim3(nblocks(off, 256)), dim3(256), 0, s, n->g, off, 0.0f);
    if (pack_all(n) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        return fail(FEDFEM_E_HIP);
    *out = n;
    return FEDFEM_OK;
}

int fedsur_destroy(fedsur_net* n) {
    destroy_net(n);
    return FEDFEM_OK;
}

int fedsur_set_stream(fedsur_net* n, void* stream) {
    if (!n) return FEDFEM_E_INVALID;
    n->stream = static_cast<hipStream_t>(stream);
    return FEDFEM_OK;
}

int fedsur_param_count(const fedsur_net* n, int64_t* count) {
    if (!n || !count) return FEDFEM_E_INVALID;
    *count = n->nparams;
    return FEDFEM_OK;
}

int fedsur_get_params(fedsur_net* n, float* host) {
    if (!n || !host) return FEDFEM_E_INVALID;
    NCHK(hipSetDevice(n->device));
    NCHK(hipMemcpyAsync(host, n->p, n->nparams * 4, hipMemcpyDeviceToHost, n->stream));
    NCHK(hipStreamSynchronize(n->stream));
    return FEDFEM_OK;
}

int fedsur_get_grads(fedsur_net* n, float* host) {
    if (!n || !host) return FEDFEM_E_INVALID;
    NCHK(hipSetDevice(n->device));
    NCHK(hipMemcpyAsync(host, n->g, n->nparams * 4, hipMemcpyDeviceToHost, n->stream));
    NCHK(hipStreamSynchronize(n->stream));
    return FEDFEM_OK;
}

int fedsur_set_params(fedsur_net* n, const float* host) {
    if (!n || !host) return FEDFEM_E_INVALID;
    for (int64_t i = 0; i < n->nparams; i++)
        if (!std::isfinite(host[i])) return FEDFEM_E_INVALID;
    NCHK(hipSetDevice(n->device));
    hipStream_t s = n->stream;
    NCHK(hipMemcpyAsync(n->p, host, n->nparams * 4, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_fill_f32, dim3(nblocks(n->nparams, 256)), dim3(256), 0, s, n->m,
                       n->nparams, 0.0f);
    hipLaunchKernelGGL(k_fill_f32, dim3(nblocks(n->nparams, 256)), dim3(256), 0, s, n->v,
                       n->nparams, 0.0f);
    n->adam_t = 0;
    NCHK(pack_all(n));
    NCHK(hipStreamSynchronize(s));
    return FEDFEM_OK;
}

int fedsur_forward(fedsur_net* n, int32_t batch, const void* x, float* y) {
    if (!n || !x || !y || batch < 1 || batch > n->Bmax) return FEDFEM_E_INVALID;
    NCHK(hipSetDevice(n->device));
    NCHK(forward_impl(n, batch, static_cast<const bf16*>(x), y));
    NCHK(hipStreamSynchronize(n->stream));
    return FEDFEM_OK;
}

int fedsur_loss_backward(fedsur_net* n, int32_t batch, const void* x, const float* target,
                         const float* mask, float* loss) {
    if (!n || !x || !target || !mask || batch < 1 || batch > n->Bmax) return FEDFEM_E_INVALID;
    NCHK(hipSetDevice(n->device));
    hipStream_t s = n->stream;
    const bf16* xb = static_cast<const bf16*>(x);
    NCHK(forward_impl(n, batch, xb, n->y));
    const int64_t V0 = vox(n, 0, batch);
    NCHK(reduce_to(n, mask, V0, n->scal));  // sum of the mask
    const int64_t nb = (V0 + 255) / 256;
    hipLaunchKernelGGL(k_mse, dim3((unsigned)nb), dim3(256), 0, s, n->y, target, mask, V0, n->scal,
                       n->dy, n->red);
    hipLaunchKernelGGL(k_colreduce, dim3(1), dim3(256), 0, s, n->red, nb, 1, n->scal + 1);
    NCHK(hipGetLastError());
    NCHK(backward_impl(n, batch, xb));
    float h[2] = {0, 0};
    NCHK(hipMemcpyAsync(h, n->scal, 8, hipMemcpyDeviceToHost, s));
    NCHK(hipStreamSynchronize(s));
    if (loss) *loss = h[0] > 0 ? h[1] / h[0] : 0.0f;
    return FEDFEM_OK;
}

int fedsur_adam_step(fedsur_net* n, float lr) {
    if (!n || !(lr > 0)) return FEDFEM_E_INVALID;
    NCHK(hipSetDevice(n->device));
    n->adam_t++;
    const float c1 = (float)(1.0 - std::pow(0.9, (double)n->adam_t));
    const float c2 = (float)(1.0 - std::pow(0.999, (double)n->adam_t));
    hipLaunchKernelGGL(k_adam, dim3(nblocks(n->nparams, 256)), dim3(256), 0, n->stream, n->p, n->g,
                       n->m, n->v, n->nparams, lr, c1, c2);
    NCHK(hipGetLastError());
    NCHK(pack_all(n));
    NCHK(hipStreamSynchronize(n->stream));
    return FEDFEM_OK;
}

int fedsur_read_activation(fedsur_net* n, int32_t layer, float* host) {
    if (!n || !host || layer < 0 || layer >= FEDSUR_LAYERS || n->B < 1) return FEDFEM_E_INVALID;
    NCHK(hipSetDevice(n->device));
    const View o = out_view(n, layer);
    const int64_t V = vox(n, o.lvl, n->B);
    float* tmp = nullptr;
    NCHK(hipMalloc(&tmp, V * o.c * 4));
    hipLaunchKernelGGL(k_bf16_to_f32, dim3(nblocks(V * o.c, 256)), dim3(256), 0, n->stream, o.p,
                       o.pitch, o.off, o.c, V, tmp);
    hipError_t e = hipMemcpyAsync(host, tmp, V * o.c * 4, hipMemcpyDeviceToHost, n->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
    (void)hipFree(tmp);
    return e == hipSuccess ? FEDFEM_OK : FEDFEM_E_HIP;
}

int fedsur_rasterize(int32_t grid, const double* frame, int32_t batch,
                     const fedsur_sample* samples, const fedsur_phys* phys, void* x, float* prior,
                     float* scale, void* stream) {
    if (grid < 1 || grid > 1024 || !frame || batch < 1 || !samples || !phys || !x || !scale)
        return FEDFEM_E_INVALID;
    if (!(frame[3] > 0) || !(phys->rho0 > 0) || !(phys->c0 > 0) || !(phys->rhob_cb >= 0) ||
        !(phys->t_heat > 0))
        return FEDFEM_E_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    RasterPhys ph{phys->rho0, phys->c0, phys->rhob_cb, phys->t_heat};
    const RasterSample* smp = reinterpret_cast<const RasterSample*>(samples);
    hipLaunchKernelGGL(k_prior_scale, dim3(nblocks(batch, 64)), dim3(64), 0, s, batch, smp, ph,
                       scale);
    const int64_t n = (int64_t)batch * grid * grid * grid;
    hipLaunchKernelGGL(k_rasterize, dim3(nblocks(n, 256)), dim3(256), 0, s, grid, frame[0],
                       frame[1], frame[2], frame[3], batch, smp, ph, scale, static_cast<bf16*>(x),
                       prior);
    return hipGetLastError() == hipSuccess ? FEDFEM_OK : FEDFEM_E_HIP;
}

int fedsur_target(int32_t grid, int32_t batch, const float* prior, const float* scale,
                  const float* T, const uint8_t* mask, float T_a, float focus, float* target,
                  float* weight, void* stream) {
    if (grid < 1 || grid > 1024 || batch < 1 || !prior || !scale || !T || !mask || !target ||
        !weight || !(focus >= 0.0f))
        return FEDFEM_E_INVALID;
    const int64_t G3 = (int64_t)grid * grid * grid;
    hipLaunchKernelGGL(k_target, dim3(nblocks(G3 * batch, 256)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), G3, batch, prior, scale, T, mask, T_a,
                       focus, target, weight);
    return hipGetLastError() == hipSuccess ? FEDFEM_OK : FEDFEM_E_HIP;
}

int fedsur_decode(int32_t grid, int32_t batch, const float* prior, const float* scale, float T_a,
                  float* y, void* stream) {
    if (grid < 1 || grid > 1024 || batch < 1 || !prior || !scale || !y) return FEDFEM_E_INVALID;
    const int64_t G3 = (int64_t)grid * grid * grid;
    hipLaunchKernelGGL(k_decode, dim3(nblocks(G3 * batch, 256)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), G3, batch, prior, scale, T_a, y);
    return hipGetLastError() == hipSuccess ? FEDFEM_OK : FEDFEM_E_HIP;
}

int fedsur_max_error(int32_t grid, int32_t batch, const float* Tp, const float* T,
                     const uint8_t* mask, float* err, void* stream) {
    if (grid < 1 || grid > 1024 || batch < 1 || batch > 65535 || !Tp || !T || !mask || !err)
        return FEDFEM_E_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t G3 = (int64_t)grid * grid * grid;
    unsigned* e = reinterpret_cast<unsigned*>(err);
    hipLaunchKernelGGL(k_fill_u32, dim3(nblocks(batch, 256)), dim3(256), 0, s, e, batch, 0u);
    const unsigned nx = (unsigned)std::min<int64_t>(64, (G3 + 255) / 256);
    hipLaunchKernelGGL(k_max_err, dim3(nx, (unsigned)batch), dim3(256), 0, s, G3, batch, Tp, T,
                       mask, e);
    return hipGetLastError() == hipSuccess ? FEDFEM_OK : FEDFEM_E_HIP;
}

int fedfem_resample(fedfem_handle* h, int32_t grid, const double* frame, float* T_out,
                    uint8_t* mask_out) {
    if (!h || grid < 1 || grid > 1024 || !frame || !T_out || !mask_out) return FEDFEM_E_INVALID;
    if (!h->precomputed) return FEDFEM_E_NOT_PRECOMPUTED;
    if (h->broken) return FEDFEM_E_HIP;
    if (!(frame[3] > 0) || h->npe != 4) return FEDFEM_E_INVALID;
    NCHK(hipSetDevice(h->device));
    hipStream_t s = h->stream;
    const int64_t nv = (int64_t)grid * grid * grid;
    int32_t* owner = nullptr;
    NCHK(hipMalloc(&owner, nv * sizeof(int32_t)));
    hipLaunchKernelGGL(k_resample_clear, dim3(nblocks(nv, 256)), dim3(256), 0, s, nv, owner, T_out,
                       mask_out);
    ResampleArgs a;
    a.E = h->E;
    a.xyz = h->d_xyz;
    a.conn = h->d_conn;
    a.T = h->d.T_[h->cur];
    a.fp32c = h->fp32c ? 1 : 0;
    a.G = grid;
    a.fx = frame[0];
    a.fy = frame[1];
    a.fz = frame[2];
    a.h = frame[3];
    a.owner = owner;
    a.out = T_out;
    a.mask = mask_out;
    hipLaunchKernelGGL(k_resample<0>, dim3(nblocks(h->E, 128)), dim3(128), 0, s, a);
    hipLaunchKernelGGL(k_resample<1>, dim3(nblocks(h->E, 128)), dim3(128), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(owner);
    return e == hipSuccess ? FEDFEM_OK : FEDFEM_E_HIP;
}

}  // extern "C"
