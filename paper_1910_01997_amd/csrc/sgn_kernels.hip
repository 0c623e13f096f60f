// HIP kernels of the surfel Gauss-Newton path for gfx950 (CDNA4).
//
// Paper: "Dense monocular SLAM by direct surfel optimization" (Trabes,
// Dondo Gazzano, Sosa Paez), Proposed Approach section, Eq. 1-10.
//
// Kernels
//   setup_kernel   per-frame constants H = K R K^-1 and K t (Eq. 6) in
//                  double; clears the work queues.
//   init_kernel    neighbour-plane initialisation (Surfel Initialization).
//   gn_kernel      the fused Gauss-Newton iterations.  A work item is a set
//                  of surfel groups inside one aligned 16 x 16-pixel block;
//                  a group fills the 64 lanes of a wavefront with pixels (four
//                  4x4 surfels or one 8x8 surfel).  Each lane loops over the
//                  neighbour frames for its pixel, with the per-pixel
//                  inverse-depth Jacobian hoisted out of the frame loop (the
//                  paper notes it does not depend on the frame); the normal
//                  equations are reduced across the surfel's lanes with DPP,
//                  and one owner lane per surfel solves its 3x3 system, all
//                  groups of the item at once.  All iterations run inside the
//                  kernel: surfels never read each other during the
//                  optimisation.
//   render_kernel  per-pixel inverse depth (and owning surfel) by Eq. 3.
//   regrid_*       surfel reference-frame change (Eq. 10) and re-gridding
//                  into another keyframe's tiles.
//   quantize_kernel  f32 images to f16 / u8 storage.
//
// Numerics.  The warp uses the closed form of Eq. 6 for a plane:
//   q = H u~ + (K t) id_u,   u_p = (q_x / q_z, q_y / q_z),
// which is K (R X + t) scaled by id_u.  id_u is formed in difference form
//   sigma = n . (r_u - r_s) / (n . r_s),   id_u = id_s (1 + sigma),
// equal to Eq. 3 without its cancellation.  The image gradient is the exact
// derivative of the bilinear interpolant.  Accumulation is in float, in a
// fixed order per surfel (frames in order per lane, then a fixed DPP tree),
// so a surfel's result depends neither on where it sits in a batch nor on
// the launch plan.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <type_traits>

#include "sgn_internal.h"
#include "surfgn.h"

namespace sgn {

// ---------------------------------------------------------------- helpers --

// Pointers into the constant address space: the descriptor tables are not
// written while a kernel runs, so uniform reads become scalar loads.
template <class T>
using cptr = const T __attribute__((address_space(4)))*;
// Global-address-space pointers (global_load with a scalar base).
template <class T>
using gptr = const T __attribute__((address_space(1)))*;
template <class T>
using gmut = T __attribute__((address_space(1)))*;

template <typename T>
__device__ __forceinline__ float ldg(gptr<T> p);
template <>
__device__ __forceinline__ float ldg<float>(gptr<float> p) { return *p; }
template <>
__device__ __forceinline__ float ldg<_Float16>(gptr<_Float16> p) { return (float)*p; }
template <>
__device__ __forceinline__ float ldg<uint8_t>(gptr<uint8_t> p) { return (float)*p; }

template <typename T>
__device__ __forceinline__ float ldpix(const T* p);
template <>
__device__ __forceinline__ float ldpix<float>(const float* p) { return *p; }
template <>
__device__ __forceinline__ float ldpix<_Float16>(const _Float16* p) { return (float)*p; }
template <>
__device__ __forceinline__ float ldpix<uint8_t>(const uint8_t* p) { return (float)*p; }

template <int CTRL>
__device__ __forceinline__ float dpp_f(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ int dpp_i(int x) {
    return __builtin_amdgcn_mov_dpp(x, CTRL, 0xF, 0xF, true);
}

// Sum over a surfel's lanes: 4 lanes (a quad), 8 (half a DPP row), 16 (one
// row), 32 (two rows) or the whole wavefront.  Every lane of the surfel ends with the
// bitwise-same value: each step adds a lane's value and its partner's, and
// float addition is commutative.
template <int LANES>
__device__ __forceinline__ float group_sum(float x) {
#pragma clang fp contract(off)
    static_assert(LANES == 4 || LANES == 8 || LANES == 16 || LANES == 32 || LANES == 64,
                  "lanes per surfel");
    x += dpp_f<0xB1>(x);
    x += dpp_f<0x4E>(x);
    if constexpr (LANES >= 8) x += dpp_f<0x141>(x);
    if constexpr (LANES >= 16) x += dpp_f<0x140>(x);
    if constexpr (LANES >= 32) x += __shfl_xor(x, 16);
    if constexpr (LANES == 64) x += __shfl_xor(x, 32);
    return x;
}
template <int LANES>
__device__ __forceinline__ int group_sum(int x) {
    static_assert(LANES == 4 || LANES == 8 || LANES == 16 || LANES == 32 || LANES == 64,
                  "lanes per surfel");
    x += dpp_i<0xB1>(x);
    x += dpp_i<0x4E>(x);
    if constexpr (LANES >= 8) x += dpp_i<0x141>(x);
    if constexpr (LANES >= 16) x += dpp_i<0x140>(x);
    if constexpr (LANES >= 32) x += __shfl_xor(x, 16);
    if constexpr (LANES == 64) x += __shfl_xor(x, 32);
    return x;
}

// Sums of two values over a surfel's lanes at once: lane 0 of the surfel
// ends with the sum of `ev`, lane 1 with the sum of `od`.  The first
// butterfly step trades halves with the neighbour lane (each lane keeps the
// value it will own and sends the other), so the remaining steps carry one
// value instead of two; they pair lanes of equal parity only (quad_perm,
// then row rotations by 4 and 8; an 8-lane surfel instead shifts its second
// quad's sums down by 4 lanes, since a rotation would bring in the
// neighbouring surfel's).  Lanes 0 and 1 form their sums in a fixed order
// that depends only on the surfel's pixels.
template <int LANES>
__device__ __forceinline__ float pair_sum(float ev, float od, bool odd) {
#pragma clang fp contract(off)
    static_assert(LANES == 4 || LANES == 8 || LANES == 16 || LANES == 32 || LANES == 64,
                  "lanes per surfel");
    const float keep = odd ? od : ev;
    const float send = odd ? ev : od;
    float x = keep + dpp_f<0xB1>(send);   // quad_perm [1,0,3,2]
    x += dpp_f<0x4E>(x);                  // quad_perm [2,3,0,1]
    if constexpr (LANES == 4) {
    } else if constexpr (LANES == 8) {
        x += dpp_f<0x104>(x);             // row_shl:4 (lane i takes lane i + 4)
    } else {
        x += dpp_f<0x124>(x);             // row_ror:4
        x += dpp_f<0x128>(x);             // row_ror:8
    }
    if constexpr (LANES >= 32) x += __shfl_xor(x, 16);
    if constexpr (LANES == 64) x += __shfl_xor(x, 32);
    return x;
}

__device__ __forceinline__ float rcp_fast(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ int find_kf(cptr<KfDev> kfs, int n_kf, int item, int hint) {
    const cptr<KfDev> h = kfs + hint;
    if (item >= h->item_base && item < h->item_base + h->n_items) return hint;
    int lo = 0, hi = n_kf - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (kfs[mid].item_base <= item) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Next work item of a persistent wavefront: take one from queue q, moving on
// to the next queue when q is exhausted; `total` when every queue is empty.
__device__ __forceinline__ int pull_item(const BatchHeader* __restrict__ hdr, uint32_t* counters,
                                         int& q, int& q_left, int lane, int total) {
    while (q_left > 0) {
        int got = 0;
        if (lane == 0) got = (int)atomicAdd(&counters[q], 1u);
        got = __builtin_amdgcn_readfirstlane(got);
        const int it = hdr->queues[q].begin + got;
        if (it < hdr->queues[q].end) return it;
        q = (q + 1 == hdr->n_queues) ? 0 : q + 1;
        --q_left;
    }
    return total;
}

// ------------------------------------------------------------ setup kernel --

// One thread per neighbour frame: H = K R K^-1 and K t in double, rounded
// once to float (Eq. 6).  Thread 0 also clears the work-queue heads.
__global__ void setup_kernel(const BatchHeader* __restrict__ hdr, uint32_t* __restrict__ counters) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kNumCounters) counters[i] = 0u;
    if (i >= hdr->n_frames) return;
    FrameDev& F = hdr->frames[i];
    // the owning keyframe carries K
    int k = 0;
    {
        int lo = 0, hi = hdr->n_kf - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (hdr->kfs[mid].frame_base <= i) lo = mid; else hi = mid - 1;
        }
        k = lo;
    }
    const KfDev& K = hdr->kfs[k];
    const double fx = K.fx_d, fy = K.fy_d, cx = K.cx_d, cy = K.cy_d;
    const double* R = F.R;
    // K R
    double KR[9];
    for (int c = 0; c < 3; ++c) {
        KR[0 * 3 + c] = fx * R[0 * 3 + c] + cx * R[2 * 3 + c];
        KR[1 * 3 + c] = fy * R[1 * 3 + c] + cy * R[2 * 3 + c];
        KR[2 * 3 + c] = R[2 * 3 + c];
    }
    // (K R) K^-1, K^-1 = [[1/fx, 0, -cx/fx], [0, 1/fy, -cy/fy], [0, 0, 1]]
    for (int r = 0; r < 3; ++r) {
        double a = KR[r * 3 + 0], b = KR[r * 3 + 1], c = KR[r * 3 + 2];
        F.hm[r * 3 + 0] = a / fx;
        F.hm[r * 3 + 1] = b / fy;
        F.hm[r * 3 + 2] = c - a * cx / fx - b * cy / fy;
    }
    F.kt[0] = fx * F.t[0] + cx * F.t[2];
    F.kt[1] = fy * F.t[1] + cy * F.t[2];
    F.kt[2] = F.t[2];
    F.zrow[0] = (float)F.hm[6];
    F.zrow[1] = (float)F.hm[7];
    F.zrow[2] = (float)F.kt[2];
    F.zrow[3] = 0.f;
}

// ------------------------------------------------------------- init kernel --

// Surfel Initialization section.  Neighbours of new surfel s: surfels that
// are not new, usable, and own a pixel closer than beta_r to u_s.  New
// id_s = mean of Eq. 3 of each neighbour's plane at r_s; new n_s = mean of
// the sign-aligned neighbour normals, renormalised.  Neighbours are visited
// in index order.
__global__ void init_kernel(const BatchHeader* __restrict__ hdr) {
    const int total = hdr->total_surfels;
    int hint = 0;
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < total; s += gridDim.x * blockDim.x) {
        int lo = 0, hi = hdr->n_kf - 1;
        if (!(s >= hdr->kfs[hint].surfel_base &&
              s < hdr->kfs[hint].surfel_base + hdr->kfs[hint].gw * hdr->kfs[hint].gh)) {
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (hdr->kfs[mid].surfel_base <= s) lo = mid; else hi = mid - 1;
            }
            hint = lo;
        }
        const KfDev& K = hdr->kfs[hint];
        if (!K.is_new) continue;
        const int S = K.patch;
        const int i = s - K.surfel_base;
        if (!K.is_new[i]) continue;
        const int gw = K.gw, gh = K.gh;
        const int tx = i % gw, ty = i / gw;
        const float half = 0.5f * (float)(S - 1);
        const float ux = (float)(S * tx) + half, uy = (float)(S * ty) + half;
        const float rsx = (ux - K.cx) / K.fx, rsy = (uy - K.cy) / K.fy;
        const float br = hdr->beta_r > 0.f ? hdr->beta_r : (float)S;
        const float br2 = br * br;
        // a tile dx columns away has its nearest pixel at |dx| S - half from
        // u_s: none beyond floor((br + half) / S) can be closer than br
        const int reach = (int)floorf((br + half) / (float)S);
        float id_sum = 0.f, sx = 0.f, sy = 0.f, sz = 0.f, rx = 0.f, ry = 0.f, rz = 0.f;
        int count = 0;
        // one neighbour tile (row ny, column nxt) in visiting order, with its
        // is_new flag, flags and state
        auto visit = [&](int ny, int nxt, uint8_t nw, uint32_t fl, float idj, float njx, float njy,
                         float njz) {
            if (nw) return;
            if (fl & (F_UNINIT | F_DEGENERATE)) return;
            // nearest pixel of tile j to the new surfel's centre
            const float qx = fminf(fmaxf(ux, (float)(S * nxt)), (float)(S * nxt + S - 1));
            const float qy = fminf(fmaxf(uy, (float)(S * ny)), (float)(S * ny + S - 1));
            const float ddx = qx - ux, ddy = qy - uy;
            if (!(ddx * ddx + ddy * ddy < br2)) return;
            const float jx = (float)(S * nxt) + half, jy = (float)(S * ny) + half;
            const float rjx = (jx - K.cx) / K.fx, rjy = (jy - K.cy) / K.fy;
            const float cj = njx * rjx + njy * rjy + njz;
            if (fabsf(cj) < 1e-6f) return;
            // Eq. 3 of plane j at ray r_s: id_j (n_j . r_s) / (n_j . r_j)
            const float id = idj * (njx * rsx + njy * rsy + njz) / cj;
            if (count == 0) { rx = njx; ry = njy; rz = njz; }
            const float sg = (njx * rx + njy * ry + njz * rz) < 0.f ? -1.f : 1.f;
            id_sum += id;
            sx += sg * njx; sy += sg * njy; sz += sg * njz;
            ++count;
        };
        if (reach == 1) {
            // the 3 x 3 neighbourhood (the default radius): every load issued
            // before the first use (out-of-grid slots read the surfel itself
            // and are skipped)
            int js[9];
            bool in[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const int ny = ty - 1 + k / 3, nxt = tx - 1 + k % 3;
                in[k] = ny >= 0 && ny < gh && nxt >= 0 && nxt < gw && k != 4;
                js[k] = in[k] ? ny * gw + nxt : i;
            }
            uint8_t nw[9];
            uint32_t fl[9];
            float idj[9], njx[9], njy[9], njz[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                nw[k] = K.is_new[js[k]];
                fl[k] = K.flags[js[k]];
                idj[k] = K.inv_depth[js[k]];
                njx[k] = K.nx[js[k]];
                njy[k] = K.ny[js[k]];
                njz[k] = K.nz[js[k]];
            }
#pragma unroll
            for (int k = 0; k < 9; ++k)
                if (in[k]) visit(ty - 1 + k / 3, tx - 1 + k % 3, nw[k], fl[k], idj[k], njx[k], njy[k], njz[k]);
        } else {
            for (int ny = ty - reach; ny <= ty + reach; ++ny) {
                if (ny < 0 || ny >= gh) continue;
                for (int nxt = tx - reach; nxt <= tx + reach; ++nxt) {
                    if (nxt < 0 || nxt >= gw) continue;
                    const int j = ny * gw + nxt;
                    if (j == i) continue;
                    visit(ny, nxt, K.is_new[j], K.flags[j], K.inv_depth[j], K.nx[j], K.ny[j], K.nz[j]);
                }
            }
        }
        if (count == 0) {
            K.flags[i] |= F_UNINIT;
            continue;
        }
        const float inv = 1.0f / (float)count;
        const float idn = id_sum * inv;
        sx *= inv; sy *= inv; sz *= inv;
        const float l2 = sx * sx + sy * sy + sz * sz;
        if (!(l2 > 0.f) || !(idn > 0.f) || !isfinite(idn) || !isfinite(l2)) {
            K.flags[i] |= F_UNINIT;
            continue;
        }
        const float il = 1.0f / sqrtf(l2);
        K.inv_depth[i] = idn;
        K.nx[i] = sx * il;
        K.ny[i] = sy * il;
        K.nz[i] = sz * il;
        K.flags[i] &= ~F_UNINIT;
    }
}

// --------------------------------------------------------------- GN kernel --

// Cholesky solve of H d = -b in double (textbook form); false when a pivot
// is <= 1e-12 max diag(H), i.e. H is not safely positive definite.
__device__ __forceinline__ bool solve3_fp64(double h00, double h01, double h02, double h11,
                                            double h12, double h22, double b0, double b1,
                                            double b2, double& d0, double& d1, double& d2) {
    const double maxd = fmax(h00, fmax(h11, h22));
    if (!(maxd > 0.0) || !isfinite(maxd)) return false;
    const double tol = 1e-12 * maxd;
    if (!(h00 > tol) || !isfinite(h00)) return false;
    const double l00 = sqrt(h00);
    const double l10 = h01 / l00, l20 = h02 / l00;
    const double p1 = h11 - l10 * l10;
    if (!(p1 > tol) || !isfinite(p1)) return false;
    const double l11 = sqrt(p1);
    const double l21 = (h12 - l20 * l10) / l11;
    const double p2 = h22 - l20 * l20 - l21 * l21;
    if (!(p2 > tol) || !isfinite(p2)) return false;
    const double l22 = sqrt(p2);
    const double y0 = -b0 / l00;
    const double y1 = (-b1 - l10 * y0) / l11;
    const double y2 = (-b2 - l20 * y0 - l21 * y1) / l22;
    d2 = y2 / l22;
    d1 = (y1 - l21 * d2) / l11;
    d0 = (y0 - l10 * d1 - l20 * d2) / l00;
    return true;
}

// Warp constants of one (anchor block, frame) pair, staged in LDS.  The
// plane-induced homography q = H u~ + (K t) id_u (Eq. 6) is evaluated in
// local coordinates: u = u_b + d, with u_b the centre of the aligned
// 16 x 16-pixel anchor block that holds the surfel and d the pixel's offset
// from it (exact, |d| <= 7.5), and an integer anchor (X0, Y0) near the block
// centre's warp at infinite depth, so that every float quantity formed per
// sample is small:
//   x_p - X0 = (Ex + hx0 dx + hx1 dy + kx id_u) / q_z
//   y_p - Y0 = (Ey + hy0 dx + hy1 dy + ky id_u) / q_z
//   q_z      =  Qz + h6 dx  + h7 dy  + k2 id_u
// with Ex = Q_x - X0 Q_z, Q = H u~_b, hx0 = h0 - X0 h6, kx = k0 - X0 k2, ...
// all formed in double once per work item and rounded once to float.  The
// block depends only on the surfel's position, so every launch plan forms
// the same words for a surfel.
constexpr int kPairWords = 12;
enum : int {
    W_HX0 = 0, W_HX1, W_KX, W_EX, W_HY0, W_HY1, W_KY, W_EY, W_QZ, W_X0, W_Y0, W_HZ1
};
// The pair words of every neighbour frame for the anchor point (qbx, qby),
// one frame per lane (lanes below nf), formed in double and rounded once,
// into the wavefront's LDS words.
__device__ __forceinline__ void stage_pair_words(const FrameDev* frames, int nf, int lane,
                                                 double qbx, double qby, float* pairs) {
    if (lane < nf) {
        const gptr<FrameDev> F = (gptr<FrameDev>)(frames + lane);
        const gptr<double> hm = F->hm;
        const gptr<double> kt = F->kt;
        const double Qx = fma(hm[0], qbx, fma(hm[1], qby, hm[2]));
        const double Qy = fma(hm[3], qbx, fma(hm[4], qby, hm[5]));
        const double Qz = fma(hm[6], qbx, fma(hm[7], qby, hm[8]));
        double X0 = 0.0, Y0 = 0.0;
        if (Qz > 0.0) {
            X0 = rint(fmin(fmax(Qx / Qz, -20000.0), 20000.0));
            Y0 = rint(fmin(fmax(Qy / Qz, -20000.0), 20000.0));
        }
        float* w = pairs + lane * kPairWords;
        w[W_HX0] = (float)(hm[0] - X0 * hm[6]);
        w[W_HX1] = (float)(hm[1] - X0 * hm[7]);
        w[W_KX] = (float)(kt[0] - X0 * kt[2]);
        w[W_EX] = (float)(Qx - X0 * Qz);
        w[W_HY0] = (float)(hm[3] - Y0 * hm[6]);
        w[W_HY1] = (float)(hm[4] - Y0 * hm[7]);
        w[W_KY] = (float)(kt[1] - Y0 * kt[2]);
        w[W_EY] = (float)(Qy - Y0 * Qz);
        w[W_QZ] = (float)Qz;
        w[W_X0] = __int_as_float((int)X0);
        w[W_Y0] = __int_as_float((int)Y0);
        w[W_HZ1] = (float)hm[7];     // h7 again, beside the words the pixel step reads
    }
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The four bilinear taps (x0, y0), (x0+1, y0), (x0, y0+1), (x0+1, y0+1) of
// one image, read with buffer loads; the second row uses the row pitch as
// the scalar offset.  f32: one 8-byte load per row.  f16 / u8: one 8-byte
// load per row from the aligned dword below the pair, and a funnel shift (4-
// and 2-byte loads at the pair's own, unaligned address measured 11 % slower
// for the whole kernel).  The tap corner is (row y0, byte column col of x0).
// Two addressings:
//  - by row (BY_ROW: every row pitch of the batch below kMaxRowStride): a
//    structured buffer whose stride is the row pitch, the row as the index
//    (range-checked against the row count) and col as the offset, so no
//    multiply forms the address;
//  - raw: the byte offset row x pitch + col, range-checked against the
//    image's bytes.
// Either way the loads run only for samples whose corner passed the validity
// test (x0 < W - 1, y0 < H - 1), so every tap lies inside the image.
struct Taps {
    float i00, i01, i10, i11;
};

typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t image_rsrc(const void* img, unsigned nbytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(img), (short)0, (int)nbytes, 0x00020000);
}
template <bool BY_ROW>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t image_rsrc_for(const void* img, unsigned pitch_b,
                                                                 unsigned rows) {
    if constexpr (BY_ROW) return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(img), (short)pitch_b, (int)rows, 0x00020000);
    else return image_rsrc(img, pitch_b * rows);
}
// buffer_load_dwordx2 ... idxen offen: base + index x stride + offset + soffset
__device__ u32x2 struct_buffer_load_b64(__amdgpu_buffer_rsrc_t rsrc, int vindex, int voffset, int soffset,
                                        int aux) __asm("llvm.amdgcn.struct.ptr.buffer.load.v2i32");
// the 8 bytes at byte column col of tap rows y0 and y0 + 1
template <bool BY_ROW>
__device__ __forceinline__ void load_row_pair(__amdgpu_buffer_rsrc_t rs, unsigned row, unsigned col,
                                              unsigned pitch_b, u32x2& a, u32x2& b) {
    if constexpr (BY_ROW) {
        a = struct_buffer_load_b64(rs, (int)row, (int)col, 0, 0);
        b = struct_buffer_load_b64(rs, (int)row, (int)col, (int)pitch_b, 0);
    } else {
        const unsigned o = __umul24(row, pitch_b) + col;
        a = __builtin_amdgcn_raw_buffer_load_b64(rs, o, 0, 0);
        b = __builtin_amdgcn_raw_buffer_load_b64(rs, o, pitch_b, 0);
    }
}
template <typename T, bool BY_ROW>
__device__ __forceinline__ Taps load_taps(__amdgpu_buffer_rsrc_t rs, unsigned row, unsigned col,
                                          unsigned pitch_b) {
    Taps t;
    u32x2 a, b;
    if constexpr (std::is_same<T, float>::value) {
        load_row_pair<BY_ROW>(rs, row, col, pitch_b, a, b);
        t.i00 = __uint_as_float(a.x);
        t.i01 = __uint_as_float(a.y);
        t.i10 = __uint_as_float(b.x);
        t.i11 = __uint_as_float(b.y);
    } else {
        // u8: the byte shift of v_alignbyte is its third operand mod 4 (the
        // pitch is a multiple of 4, so col's shift is the address's)
        load_row_pair<BY_ROW>(rs, row, col & ~3u, pitch_b, a, b);
        const unsigned pa = __builtin_amdgcn_alignbyte(a.y, a.x, col);
        const unsigned pb = __builtin_amdgcn_alignbyte(b.y, b.x, col);
        t.i00 = (float)(pa & 0xffu);
        t.i01 = (float)((pa >> 8) & 0xffu);
        t.i10 = (float)(pb & 0xffu);
        t.i11 = (float)((pb >> 8) & 0xffu);
    }
    return t;
}

// The two row interpolants of a bilinear sample: for each tap row the
// difference d = I(x0+1) - I(x0) and the value I(x0) + ax d.  f32 and u8
// decode the taps first; f16 works on the packed pair directly with mixed
// precision FMAs (the halves convert exactly to float, so the rounding is
// that of the float form).
struct Lerp {
    float d0, top, d1, bot;
};

template <typename T, bool BY_ROW>
__device__ __forceinline__ Lerp lerp_rows(__amdgpu_buffer_rsrc_t rs, unsigned row, unsigned col, unsigned pitch_b,
                                          float ax) {
    const Taps t = load_taps<T, BY_ROW>(rs, row, col, pitch_b);
    Lerp l;
    l.d0 = t.i01 - t.i00;
    l.d1 = t.i11 - t.i10;
    l.top = fmaf(ax, l.d0, t.i00);
    l.bot = fmaf(ax, l.d1, t.i10);
    return l;
}

// hi - lo of a packed pair of halves, in float
__device__ __forceinline__ float half_pair_diff(unsigned pk) {
    float r;
    asm("v_fma_mix_f32 %0, %1, 1.0, -%1 op_sel:[1,0,0] op_sel_hi:[1,0,1]" : "=v"(r) : "v"(pk));
    return r;
}
// a * b + lo (the low half of pk), in float
__device__ __forceinline__ float half_lo_fma(float a, float b, unsigned pk) {
    float r;
    asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel_hi:[0,0,1]" : "=v"(r) : "v"(a), "v"(b), "v"(pk));
    return r;
}

template <bool BY_ROW>
__device__ __forceinline__ Lerp lerp_rows_f16(__amdgpu_buffer_rsrc_t rs, unsigned row, unsigned col,
                                              unsigned pitch_b, float ax) {
    // pitch_b is a multiple of 4; the byte funnel shift (v_alignbyte) takes
    // its amount mod 4, so col gives the address's shift
    u32x2 va, vb;
    load_row_pair<BY_ROW>(rs, row, col & ~3u, pitch_b, va, vb);
    const unsigned a = __builtin_amdgcn_alignbyte(va.y, va.x, col);  // (I(x0), I(x0+1)) of row y0
    const unsigned b = __builtin_amdgcn_alignbyte(vb.y, vb.x, col);  // of row y0 + 1
    Lerp l;
    l.d0 = half_pair_diff(a);
    l.d1 = half_pair_diff(b);
    l.top = half_lo_fma(ax, l.d0, a);
    l.bot = half_lo_fma(ax, l.d1, b);
    return l;
}

template <typename T, bool BY_ROW>
__device__ __forceinline__ Lerp sample_rows(__amdgpu_buffer_rsrc_t rs, unsigned row, unsigned col,
                                            unsigned pitch_b, float ax) {
    if constexpr (std::is_same<T, _Float16>::value) return lerp_rows_f16<BY_ROW>(rs, row, col, pitch_b, ax);
    else return lerp_rows<T, BY_ROW>(rs, row, col, pitch_b, ax);
}

// floor(x) converted to int in one instruction (v_cvt_flr_i32_f32).
__device__ __forceinline__ int cvt_floor(float x) {
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// Warp of one sample into frame f in local coordinates (see the pair words):
// returns validity; on success the integer tap corner (row, col) and the
// bilinear fractions.  Valid iff q_z > 0 and 0 <= x_p < W-1, 0 <= y_p < H-1,
// decided exactly on the integer corner X0 + floor(x_p - X0).
struct Warp {
    float fx, fy, rq, ax, ay;
    unsigned row, col;          // tap corner: row y0, byte column of x0
    bool v;
};

template <typename T>
__device__ __forceinline__ Warp warp_sample(const float4& c0, const float4& c1, const float4& c2,
                                            float h6, float h7, float k2, float dx, float dy,
                                            float idu, bool pix_ok, unsigned wm1, unsigned hm1,
                                            unsigned pitch_b) {
    Warp w;
    const float nxq = fmaf(c0.x, dx, fmaf(c0.y, dy, fmaf(c0.z, idu, c0.w)));
    const float nyq = fmaf(c1.x, dx, fmaf(c1.y, dy, fmaf(c1.z, idu, c1.w)));
    const float qz = fmaf(h6, dx, fmaf(h7, dy, fmaf(k2, idu, c2.x)));
    w.rq = rcp_fast(qz);
    w.fx = nxq * w.rq;                                   // x_p - X0
    w.fy = nyq * w.rq;                                   // y_p - Y0
    const int flx = cvt_floor(w.fx), fly = cvt_floor(w.fy);
    // unsigned wrap-around: out-of-range (or saturated) corners fail the test
    const unsigned ix = __float_as_uint(c2.y) + (unsigned)flx;
    const unsigned iy = __float_as_uint(c2.z) + (unsigned)fly;
    w.v = pix_ok & (qz > 0.f) & (ix < wm1) & (iy < hm1);
    w.ax = __builtin_amdgcn_fractf(w.fx);
    w.ay = __builtin_amdgcn_fractf(w.fy);
    w.row = iy; w.col = ix * (unsigned)sizeof(T);
    return w;
}

// The frame loop of one Gauss-Newton iteration for one pixel (lane): warp
// into every neighbour frame, bilinear sample with gradient, Huber-weighted
// residual, and the scalar chain factor a = dr/did_u.  Accumulates
// A = sum w a^2 and B = sum w a r (the per-pixel Jacobian g is applied after
// the loop, hoisted as the paper suggests).  LAST also sums the Huber cost.
template <typename T, bool LAST, bool BY_ROW>
__device__ __forceinline__ void frame_loop(const float* __restrict__ pc, cptr<FrameDev> fr, int nf,
                                           float dx, float dy, float idu, bool pix_ok,
                                           unsigned pitch_b, unsigned img_bytes, unsigned wm1,
                                           unsigned hm1, float ikf, float hk, float img_scale,
                                           float& A, float& B, float& cst, int& nvl) {
    constexpr bool SCALED = std::is_same<T, uint8_t>::value;
    for (int f = 0; f < nf; ++f) {
        const float4 c0 = *(const float4*)(pc + f * kPairWords);
        const float4 c1 = *(const float4*)(pc + f * kPairWords + 4);
        const float4 c2 = *(const float4*)(pc + f * kPairWords + 8);
        const float h6 = fr[f].zrow[0], h7 = fr[f].zrow[1], k2 = fr[f].zrow[2];
        const __amdgpu_buffer_rsrc_t rs = image_rsrc_for<BY_ROW>(fr[f].img, pitch_b, hm1 + 1);
        // Eq. 6 in local coordinates
        const Warp w = warp_sample<T>(c0, c1, c2, h6, h7, k2, dx, dy, idu, pix_ok, wm1, hm1, pitch_b);
        if (w.v) {
            const Lerp l = sample_rows<T, BY_ROW>(rs, w.row, w.col, pitch_b, w.ax);
            // bilinear value and the exact gradient of the interpolant
            const float gy = l.bot - l.top;
            const float val = fmaf(w.ay, gy, l.top);
            const float gx = fmaf(w.ay, l.d1 - l.d0, l.d0);
            // residual (Eq. 5) and Huber IRLS weight w = min(1, k/|r|) (Eq. 8)
            const float r = SCALED ? fmaf(val, img_scale, -ikf) : val - ikf;
            const float ar = fabsf(r);
            // (the clamp to [0, 1] folds into the multiply; it maps a NaN
            // weight to 0 where min(1, NaN) gives 1, which changes nothing
            // the update reports: B = sum w a r is NaN either way)
            const float wt = fminf(fmaxf(hk * rcp_fast(ar), 0.f), 1.f);
            // dr/did_u = grad I . dpi/dq . K t  (Eq. 8 with dq/did_u = K t):
            // (k0 - x_p k2) = kx - (x_p - X0) k2, likewise for y
            const float tx_ = fmaf(-w.fx, k2, c0.z);
            const float ty_ = fmaf(-w.fy, k2, c1.z);
            const float a = fmaf(gx, tx_, gy * ty_) * (SCALED ? w.rq * img_scale : w.rq);
            const float wa = wt * a;
            A = fmaf(wa, a, A);
            B = fmaf(wa, r, B);
            ++nvl;
            if constexpr (LAST) cst += (ar <= hk) ? 0.5f * r * r : hk * (ar - 0.5f * hk);
        }
    }
}

// One sample from its homogeneous warp q = (nxq, nyq, qz) in local
// coordinates (see the pair words): validity on the integer corner, the
// bilinear value and exact gradient, residual, Huber IRLS weight and chain
// factor; accumulates A, B, the valid count and (LAST) the Huber cost.
template <typename T, bool LAST, bool BY_ROW>
__device__ __forceinline__ void sample_at(float nxq, float nyq, float qz, const float4& c0, const float4& c1,
                                          const float4& c2, float k2, __amdgpu_buffer_rsrc_t rs, bool pix_ok,
                                          unsigned pitch_b, unsigned wm1, unsigned hm1, float ikf, float hk,
                                          float img_scale, float& A, float& B, float& cst, unsigned& nvl,
                                          unsigned one = 1u) {
    constexpr bool SCALED = std::is_same<T, uint8_t>::value;
    const float rq = rcp_fast(qz);
    const float fx = nxq * rq;                            // x_p - X0
    const float fy = nyq * rq;                            // y_p - Y0
    const int flx = cvt_floor(fx), fly = cvt_floor(fy);
    // unsigned wrap-around: out-of-range (or saturated) corners fail the test
    const unsigned ix = __float_as_uint(c2.y) + (unsigned)flx;
    const unsigned iy = __float_as_uint(c2.z) + (unsigned)fly;
    if (pix_ok & (qz > 0.f) & (ix < wm1) & (iy < hm1)) {
        const float ax = __builtin_amdgcn_fractf(fx);
        const float ay = __builtin_amdgcn_fractf(fy);
        const Lerp l = sample_rows<T, BY_ROW>(rs, iy, ix * (unsigned)sizeof(T), pitch_b, ax);
        // bilinear value and the exact gradient of the interpolant
        const float gy = l.bot - l.top;
        const float val = fmaf(ay, gy, l.top);
        const float gx = fmaf(ay, l.d1 - l.d0, l.d0);
        // residual (Eq. 5) and Huber IRLS weight w = min(1, k/|r|) (Eq. 8)
        const float r = SCALED ? fmaf(val, img_scale, -ikf) : val - ikf;
        const float ar = fabsf(r);
        // (the clamp to [0, 1] folds into the multiply; it maps a NaN weight
        // to 0 where min(1, NaN) gives 1, which changes nothing the update
        // reports: B = sum w a r is NaN either way)
        const float wt = fminf(fmaxf(hk * rcp_fast(ar), 0.f), 1.f);
        // dr/did_u = grad I . dpi/dq . K t  (Eq. 8 with dq/did_u = K t):
        // (k0 - x_p k2) = kx - (x_p - X0) k2, likewise for y
        const float tx_ = fmaf(-fx, k2, c0.z);
        const float ty_ = fmaf(-fy, k2, c1.z);
        const float a = fmaf(gx, tx_, gy * ty_) * (SCALED ? rq * img_scale : rq);
        const float wa = wt * a;
        A = fmaf(wa, a, A);
        B = fmaf(wa, r, B);
        nvl += one;
        if constexpr (LAST) cst += (ar <= hk) ? 0.5f * r * r : hk * (ar - 0.5f * hk);
    }
}

// The frame loop for the NP pixels of one lane at once: for each neighbour
// frame the frame's constants are read once, the first pixel's warp is
// formed from its offset (dx, dy) from the anchor block centre and its
// inverse depth idu0, and the others' incrementally: pixel j lies dyr rows
// below pixel j-1 of the same surfel and its id_u is didu larger (id_u is
// affine along the column), so its q adds the frame's step, dyr times the
// homography's y column plus didu times K t.  Accumulates A, B and the cost
// per pixel as frame_loop does; the valid counts of the pixels are packed
// one per byte of nvp (pixel j in byte j; at most 16 frames each).
template <typename T, bool LAST, int NP, bool BY_ROW>
__device__ __forceinline__ void frame_loop_px(const float* __restrict__ pc, cptr<FrameDev> fr, int nf,
                                              float dx, float dy, float dyr, float idu0, float didu,
                                              const bool (&pix_ok)[NP],
                                              unsigned pitch_b, unsigned img_bytes, unsigned wm1,
                                              unsigned hm1, const float (&ikf)[NP], float hk, float img_scale,
                                              float (&A)[NP], float (&B)[NP], float (&cst)[NP],
                                              unsigned& nvp) {
    static_assert(NP <= 4, "four byte counters");
    for (int f = 0; f < nf; ++f) {
        const float4 c0 = *(const float4*)(pc + f * kPairWords);
        const float4 c1 = *(const float4*)(pc + f * kPairWords + 4);
        const float4 c2 = *(const float4*)(pc + f * kPairWords + 8);
        const float h6 = fr[f].zrow[0], h7 = fr[f].zrow[1], k2 = fr[f].zrow[2];
        const __amdgpu_buffer_rsrc_t rs = image_rsrc_for<BY_ROW>(fr[f].img, pitch_b, hm1 + 1);
        // Eq. 6 in local coordinates
        float nxq = fmaf(c0.x, dx, fmaf(c0.y, dy, fmaf(c0.z, idu0, c0.w)));
        float nyq = fmaf(c1.x, dx, fmaf(c1.y, dy, fmaf(c1.z, idu0, c1.w)));
        float qz = fmaf(h6, dx, fmaf(h7, dy, fmaf(k2, idu0, c2.x)));
        sample_at<T, LAST, BY_ROW>(nxq, nyq, qz, c0, c1, c2, k2, rs, pix_ok[0], pitch_b, wm1, hm1, ikf[0], hk,
                           img_scale, A[0], B[0], cst[0], nvp, 1u);
        if constexpr (NP > 1) {
            const float sx = fmaf(c0.z, didu, c0.y * dyr);
            const float sy = fmaf(c1.z, didu, c1.y * dyr);
            const float sz = fmaf(k2, didu, c2.w * dyr);     // c2.w = h7
#pragma unroll
            for (int j = 1; j < NP; ++j) {
                nxq += sx;
                nyq += sy;
                qz += sz;
                sample_at<T, LAST, BY_ROW>(nxq, nyq, qz, c0, c1, c2, k2, rs, pix_ok[j], pitch_b, wm1, hm1, ikf[j],
                                   hk, img_scale, A[j], B[j], cst[j], nvp, 1u << (8 * j));
            }
        }
    }
}

// Huber cost (Eq. 5) and valid-sample count of one pixel at a candidate
// state, over all neighbour frames (no Jacobian): the Levenberg-Marquardt
// acceptance test.
template <typename T, bool BY_ROW>
__device__ __forceinline__ void frame_cost(const float* __restrict__ pc, cptr<FrameDev> fr, int nf,
                                           float dx, float dy, float idu, bool pix_ok,
                                           unsigned pitch_b, unsigned img_bytes, unsigned wm1,
                                           unsigned hm1, float ikf, float hk, float img_scale,
                                           float& cst, int& nvl) {
    constexpr bool SCALED = std::is_same<T, uint8_t>::value;
    for (int f = 0; f < nf; ++f) {
        const float4 c0 = *(const float4*)(pc + f * kPairWords);
        const float4 c1 = *(const float4*)(pc + f * kPairWords + 4);
        const float4 c2 = *(const float4*)(pc + f * kPairWords + 8);
        const float h6 = fr[f].zrow[0], h7 = fr[f].zrow[1], k2 = fr[f].zrow[2];
        const __amdgpu_buffer_rsrc_t rs = image_rsrc_for<BY_ROW>(fr[f].img, pitch_b, hm1 + 1);
        const Warp w = warp_sample<T>(c0, c1, c2, h6, h7, k2, dx, dy, idu, pix_ok, wm1, hm1, pitch_b);
        if (w.v) {
            const Lerp l = sample_rows<T, BY_ROW>(rs, w.row, w.col, pitch_b, w.ax);
            const float val = fmaf(w.ay, l.bot - l.top, l.top);
            const float r = SCALED ? fmaf(val, img_scale, -ikf) : val - ikf;
            const float ar = fabsf(r);
            cst += (ar <= hk) ? 0.5f * r * r : hk * (ar - 0.5f * hk);
            ++nvl;
        }
    }
}

// Per-surfel records exchanged through LDS between the pixel lanes and the
// surfel's owner lane (see gn_kernel).
enum : int {
    // state broadcast to the pixel lanes
    ST_ID = 0, ST_NX, ST_NY, ST_NZ, ST_B1X, ST_B1Y, ST_B1Z, ST_B2X, ST_B2Y, ST_B2Z, ST_INVC,
    ST_RSX, ST_RSY, ST_ALIVE,
    // the owner's own bookkeeping, parked here through the group loop
    ST_FLAGS, ST_LAM, ST_COSTO, ST_NVO, ST_WORDS = 20
};
enum : int {
    // reduced normal equations sent to the owner
    SM_H00 = 0, SM_H01, SM_H02, SM_H11, SM_H12, SM_H22, SM_B0, SM_B1, SM_B2, SM_NV, SM_COST,
    SM_WORDS = 12
};
constexpr int kMaxItemSurfels = 16;

// Tangent basis of n: b1 = normalise(e - (e.n) n), e = x^ if |n_x| < 0.9
// else y^, and b2 = n x b1.
__device__ __forceinline__ void tangent_basis(float nx, float ny, float nz, float& b1x, float& b1y,
                                              float& b1z, float& b2x, float& b2y, float& b2z) {
    const bool ex = fabsf(nx) < 0.9f;
    const float en = ex ? nx : ny;
    b1x = (ex ? 1.f : 0.f) - en * nx;
    b1y = (ex ? 0.f : 1.f) - en * ny;
    b1z = -en * nz;
    const float ib = __frsqrt_rn(b1x * b1x + b1y * b1y + b1z * b1z);
    b1x *= ib; b1y *= ib; b1z *= ib;
    b2x = ny * b1z - nz * b1y;
    b2y = nz * b1x - nx * b1z;
    b2z = nx * b1y - ny * b1x;
}

// One Gauss-Newton step of a surfel on its owner lane, from the reduced
// normal equations sm[] (J^T W J, J^T W r, valid count and cost, laid out as
// SM_*): FEW_SAMPLES below three samples; otherwise the equilibrated 3 x 3
// system (diagonal scaled by 1 + lam) is solved in float by its adjugate, or
// in double by Cholesky when its Frobenius condition exceeds kappa_fp64 or a
// pivot is not safely positive; then id_s += d0 and n = normalise(n + d1 b1 +
// d2 b2) (id_s alone for the depth-only ablation).  Returns true with the
// candidate state when a step is proposed; sets the flags otherwise (a
// rejected step raises lam tenfold when damping is on).
__device__ __forceinline__ bool owner_step(const float* sm, bool alive, bool last,
                                           bool depth_only, bool lm, float kap2, float& lam,
                                           float id, float nx, float ny, float nz, float b1x,
                                           float b1y, float b1z, float b2x, float b2y, float b2z,
                                           uint32_t& flags, float& cost_out, int& nv_out, int& nv,
                                           float& cost_here, float& id_c, float& nx_c,
                                           float& ny_c, float& nz_c) {
    bool cand = false;
    const float H00 = sm[SM_H00], H01 = sm[SM_H01], H02 = sm[SM_H02];
    const float H11 = sm[SM_H11], H12 = sm[SM_H12], H22 = sm[SM_H22];
    const float bb0 = sm[SM_B0], bb1 = sm[SM_B1], bb2 = sm[SM_B2];
    nv = (int)sm[SM_NV];
    cost_here = sm[SM_COST];
    if (alive && last) cost_out = cost_here;
    if (alive) {
        nv_out = nv;
        float d0s = 0.f, d1s = 0.f, d2s = 0.f;
        bool ok = true;
        if (nv < 3) {
            flags |= F_FEW_SAMPLES;
            ok = false;
        }
        const float dd = 1.f + lam;          // (H + lam diag H): equilibrated diagonal
        if (ok && depth_only) {
            if (H00 > 0.f && isfinite(H00)) {
                d0s = -bb0 * rcp_fast(H00 * dd);
            } else {
                flags |= F_SOLVE_FAIL;
                ok = false;
            }
        } else if (ok) {
            // equilibrate: E = D^-1/2 H D^-1/2 (unit diagonal).  The float
            // solve is formed unconditionally (no branches: the tests below
            // are combined with |) and replaced by the double-precision one
            // where a diagonal is not positive and finite or the system is
            // too ill-conditioned for float.
            const float maxd = fmaxf(H00, fmaxf(H11, H22));
            const float e0 = __frsqrt_rn(H00), e1 = __frsqrt_rn(H11), e2 = __frsqrt_rn(H22);
            const float e01 = H01 * e0 * e1, e02 = H02 * e0 * e2, e12 = H12 * e1 * e2;
            // adjugate and determinant of E (diagonal dd = 1 + lambda)
            const float d2 = dd * dd;
            const float c00 = fmaf(-e12, e12, d2), c11 = fmaf(-e02, e02, d2);
            const float c22 = fmaf(-e01, e01, d2);
            const float c01 = fmaf(e02, e12, -dd * e01), c02 = fmaf(e01, e12, -dd * e02);
            const float c12 = fmaf(e01, e02, -dd * e12);
            const float det = fmaf(e01, c01, fmaf(e02, c02, dd * c00));
            // kappa_F(E)^2 = ||E||_F^2 ||adj E||_F^2 / det^2  (>= kappa_2(E)^2)
            const float fro2 = 3.f * d2 + 2.f * (e01 * e01 + e02 * e02 + e12 * e12);
            const float adj2 = c00 * c00 + c11 * c11 + c22 * c22 +
                               2.f * (c01 * c01 + c02 * c02 + c12 * c12);
            // raw Cholesky pivots are H_jj times the equilibrated ones
            const float p1 = c22 * rcp_fast(dd);   // dd - e01^2 / dd (only compared)
            const float p2 = det * rcp_fast(c22);  // (only compared)
            const bool need64 = !(H00 > 0.f) | !(H11 > 0.f) | !(H22 > 0.f) | !isfinite(maxd) |
                                !(fro2 * adj2 <= kap2 * det * det) | !(det > 0.f) | !(c22 > 0.f) |
                                !(H11 * p1 > 1e-10f * maxd * dd) | !(H22 * p2 > 1e-10f * maxd * dd);
            {
                const float bh0 = bb0 * e0, bh1 = bb1 * e1, bh2 = bb2 * e2;
                const float idet = rcp_fast(det);
                d0s = -(c00 * bh0 + c01 * bh1 + c02 * bh2) * idet * e0;
                d1s = -(c01 * bh0 + c11 * bh1 + c12 * bh2) * idet * e1;
                d2s = -(c02 * bh0 + c12 * bh1 + c22 * bh2) * idet * e2;
            }
            if (need64) {
                flags |= F_FP64_SOLVE;
                double dd0 = 0.0, dd1 = 0.0, dd2 = 0.0;
                const double dmp = 1.0 + (double)lam;
                if (solve3_fp64((double)H00 * dmp, H01, H02, (double)H11 * dmp, H12,
                                (double)H22 * dmp, bb0, bb1, bb2, dd0, dd1, dd2)) {
                    d0s = (float)dd0; d1s = (float)dd1; d2s = (float)dd2;
                } else {
                    flags |= F_SOLVE_FAIL;
                    ok = false;
                }
            }
        }
        if (ok) {
            // update: id_s += d0; n = normalise(n + d1 b1 + d2 b2) (the
            // depth-only ablation moves id_s alone and keeps n)
            id_c = id + d0s;
            nx_c = nx; ny_c = ny; nz_c = nz;
            bool ok_step;
            if (depth_only) {
                ok_step = (id_c > 0.f) && isfinite(id_c);
            } else {
                const float mx = fmaf(d1s, b1x, fmaf(d2s, b2x, nx));
                const float my = fmaf(d1s, b1y, fmaf(d2s, b2y, ny));
                const float mz = fmaf(d1s, b1z, fmaf(d2s, b2z, nz));
                const float l2 = mx * mx + my * my + mz * mz;
                ok_step = (id_c > 0.f) && isfinite(id_c) && (l2 > 0.f) && isfinite(l2);
                if (ok_step) {
                    const float il = __frsqrt_rn(l2);
                    nx_c = mx * il; ny_c = my * il; nz_c = mz * il;
                }
            }
            if (!ok_step) {
                flags |= F_REJECTED;
                if (lm) lam *= 10.f;
            } else {
                cand = true;
            }
        }
    }
    return cand;
}

// Levenberg-Marquardt acceptance of a candidate on its owner lane: the
// candidate's cost cost2 over nv2 valid samples against the current cost
// over nv.  Accepted when the mean Huber cost per valid sample does not rise
// (cost2 / nv2 <= cost / nv, compared as cost2 nv <= cost nv2) and at least
// three samples remain.  lam shrinks tenfold (floor 1e-9) on acceptance and
// grows tenfold on refusal.
__device__ __forceinline__ bool lm_accept(float cost2, int nv2, float cost_here, int nv, float& lam) {
    if (nv2 < 3 || !(cost2 * (float)nv <= cost_here * (float)nv2)) {
        lam *= 10.f;
        return false;
    }
    lam = fmaxf(lam * 0.1f, 1e-9f);
    return true;
}

// The fused Gauss-Newton kernel.
//
// Mapping.  A work item is a block of surfels inside one aligned anchor
// block (16 x 16 pixels): K groups, each filling the 64 lanes of the
// wavefront with pixels (S = 4: a TX x TY arrangement of four, eight or
// sixteen 4 x 4 surfels, 16, 8 or 4 lanes per surfel, one, two or four
// pixels per lane; S = 8: one 8 x 8 surfel; S = 16: one 16 x 16 surfel,
// four pixels per lane).  Per iteration the wavefront walks its groups; for
// each, every lane forms the frame-independent terms of its pixels' surfel
// (hoisted as the paper suggests), loops over the neighbour frames (warp,
// bilinear sample and gradient, Huber-weighted residual, chain factor) and
// the surfel's lanes reduce J^T W J and J^T W r with DPP.  Each surfel has
// an owner lane (lane k among the surfel's lanes for group k); the owners
// then solve all K groups' 3 x 3 systems at once, so the per-surfel work
// (solve, update, tangent basis) is issued once per K groups.  Sums and states pass
// between the pixel lanes and the owners through LDS.  All iterations run in
// the kernel: surfels never read each other during the optimisation.
// Registers are the budget that matters (the kernel issues a VALU
// instruction on nearly every cycle it can, and more wavefronts per SIMD
// hide the rest): values that the frame loop does not use are not held
// through it but formed again or read back from LDS afterwards.  BY_ROW
// reads the neighbour rows by index (row pitches below kMaxRowStride).
//
// Wavefronts per SIMD each plan's kernel is compiled for (the register
// budget: 72 VGPRs for seven, 80 for six, 96 for five).  Occupancy pays: on
// the 64-keyframe f16 batch the 4x4 one-group kernel takes 4.69 ms at four,
// 4.30 at five, 3.94 at six and 3.76 at seven (its 11-12 spilled words are
// stored and reloaded once per work item, or in the damped variant's
// branches); at eight, with spills inside the iteration loop, 4.05 ms.
template <int S, int K>
constexpr int gn_waves() { return K == 1 ? 7 : (S == 8 ? 6 : 5); }

template <typename T, int S, int TX, int TY, int K, bool BY_ROW>
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(gn_waves<S, K>(), 8))) void gn_kernel(const BatchHeader* __restrict__ hdr_,
                                                           uint32_t* __restrict__ counters,
                                                           int persistent) {
    constexpr ItemGeo G = item_geo(S, TX, TY, K);
    constexpr int PIX = S * S;                                // pixels per surfel
    constexpr int SLOTS = TX * TY;                            // surfels per group
    constexpr int LANES = kWaveSize / SLOTS;                  // lanes per surfel
    constexpr int PPL = PIX / LANES;                          // pixels per lane
    constexpr int NS = K * SLOTS;                             // surfels per work item
    constexpr float DYR = (float)(LANES / S);                 // rows between a lane's pixels
    static_assert(PPL * LANES == PIX, "a group fills the wavefront");
    static_assert(PPL == 1 || LANES % S == 0, "a lane's pixels share a column");
    static_assert(NS <= kMaxItemSurfels && K <= LANES, "surfels per item");
    static_assert(G.ix <= G.ab && G.iy <= G.ab, "a work item lies in one anchor block");
    const cptr<BatchHeader> hdr = (cptr<BatchHeader>)hdr_;
    const int lane = threadIdx.x & (kWaveSize - 1);
    const int wave = threadIdx.x >> 6;
    // pixel role: slot r of a group; pixels p + LANES j (j < PPL) of that surfel
    const int r = lane / LANES;
    const int p = lane % LANES;
    const float half = 0.5f * (float)(S - 1);
    int pxs[PPL], pys[PPL];
    float dxp[PPL], dyp[PPL];                    // offsets from u_s (exact)
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
        const int q = p + LANES * j;
        pxs[j] = q % S;
        pys[j] = q / S;
        dxp[j] = (float)pxs[j] - half;
        dyp[j] = (float)pys[j] - half;
    }
    // owner role: surfel (group ok_g, slot ok_r) of the item
    const int ok_g = SLOTS == 1 ? lane : lane & (LANES - 1);
    const int ok_r = SLOTS == 1 ? 0 : lane >> __builtin_ctz(LANES);
    const bool owner = ok_g < K;
    const int own = ok_g * SLOTS + ok_r;

    const int n_kf = hdr->n_kf;
    const int total = hdr->total_items;
    const int iters = hdr->iters;
    const float hk = hdr->huber_k;
    const float kappa_s = hdr->kappa_fp64;
    const bool depth_only = hdr->depth_only != 0;
    const uint32_t stamp = hdr->stamp;
    const float lm0 = hdr->lm_lambda;
    const bool lm = lm0 > 0.f;
    const cptr<KfDev> kfs = (cptr<KfDev>)hdr->kfs;

    __shared__ float4 s_pairs[kBlockThreads / kWaveSize][kMaxNbr * kPairWords / 4];
    __shared__ float4 s_state[kBlockThreads / kWaveSize][kMaxItemSurfels * ST_WORDS / 4];
    __shared__ float4 s_sums[kBlockThreads / kWaveSize][kMaxItemSurfels * SM_WORDS / 4];
    float* const pairs = (float*)s_pairs[wave];
    float* const lst = (float*)s_state[wave];
    float* const lsm = (float*)s_sums[wave];

    int q = persistent ? (int)(blockIdx.x % (unsigned)kXcds) % hdr->n_queues : 0;
    int q_left = hdr->n_queues;
    int hint = 0;
    int item;
    if (persistent) {
        item = pull_item(hdr_, counters, q, q_left, lane, total);
    } else if (hdr->n_queues == kXcds) {
        // one share of the work items per XCD: the hardware hands the
        // workgroups to the XCDs in turn, so workgroup b runs on XCD
        // b % kXcds and takes that share's items in order (every item is
        // still taken once under any other dispatch order; only the L2
        // locality depends on it)
        const int share = (int)(blockIdx.x % (unsigned)kXcds);
        const int it = hdr->queues[share].begin +
                       (int)(blockIdx.x / (unsigned)kXcds) * (kBlockThreads / kWaveSize) + wave;
        item = it < hdr->queues[share].end ? it : total;
    } else {
        item = blockIdx.x * (kBlockThreads / kWaveSize) + wave;
    }
    for (; item < total;
         item = persistent ? pull_item(hdr_, counters, q, q_left, lane, total) : total) {
        item = __builtin_amdgcn_readfirstlane(item);
        const int kidx = find_kf(kfs, n_kf, item, hint);
        hint = kidx;
        const cptr<KfDev> Kd = kfs + kidx;
        // item -> anchor block (bx, by) and the item's place in it
        const int g = item - Kd->item_base;
        const int blk = g / G.ipb, sub = g - blk * G.ipb;
        const int bx = blk % Kd->groups_x, by = blk / Kd->groups_x;
        const int it0x = bx * G.ab + (sub % (G.ab / G.ix)) * G.ix;
        const int it0y = by * G.ab + (sub / (G.ab / G.ix)) * G.iy;
        const int gw = Kd->gw, gh = Kd->gh;
        if (it0x >= gw || it0y >= gh) continue;          // item entirely outside the grid
        const int nf = Kd->n_nbr;
        const float img_scale = Kd->img_scale;
        const unsigned pitch_b = (unsigned)Kd->nbr_pitch_b;
        const unsigned img_bytes = pitch_b * (unsigned)Kd->height;
        const unsigned wm1 = (unsigned)(Kd->width - 1), hm1 = (unsigned)(Kd->height - 1);
        const float fxk = Kd->fx, fyk = Kd->fy, cxk = Kd->cx, cyk = Kd->cy;
        // r_u - r_s of the lane's first pixel; its later pixels lie DYR rows
        // apart in the same column, dyr_f apart in r
        const float drx0 = dxp[0] / fxk, dry0 = dyp[0] / fyk;
        const float dyr_f = DYR / fyk;
        // anchor block centre (pixels)
        const int bpx = bx * G.ab * S, bpy = by * G.ab * S;
        {
            // warp constants of every frame for this anchor block, one frame
            // per lane, in double
            wave_sync();
            stage_pair_words(hdr->frames + Kd->frame_base, nf, lane,
                             (double)bpx + 0.5 * (double)(G.ab * S - 1),
                             (double)bpy + 0.5 * (double)(G.ab * S - 1), pairs);
        }
        // the frame table pointer is wave-uniform: keep it in SGPRs
        const uint64_t fr_bits = (uint64_t)(const void*)(hdr->frames + Kd->frame_base);
        const uint32_t fr_lo = __builtin_amdgcn_readfirstlane((uint32_t)fr_bits);
        const uint32_t fr_hi = __builtin_amdgcn_readfirstlane((uint32_t)(fr_bits >> 32));
        const cptr<FrameDev> fr = (cptr<FrameDev>)(((uint64_t)fr_hi << 32) | fr_lo);

        // pixel lanes: keyframe value of this lane's pixels in every group
        float ikf[K][PPL];
        const gptr<T> kimg = (gptr<T>)Kd->kf_img;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int tx = it0x + (k % G.gx) * TX + r % TX, ty = it0y + (k / G.gx) * TY + r / TX;
#pragma unroll
            for (int j = 0; j < PPL; ++j) {
                ikf[k][j] = 0.f;
                if (tx < gw && ty < gh)
                    ikf[k][j] = ldg<T>(kimg + ((unsigned)(S * ty + pys[j]) * (unsigned)Kd->kf_pitch +
                                               (unsigned)(S * tx + pxs[j]))) * Kd->kf_scale;
            }
        }

        // owner lanes: the surfel's state
        const int otx = it0x + (ok_g % G.gx) * TX + ok_r % TX;
        const int oty = it0y + (ok_g / G.gx) * TY + ok_r / TX;
        const bool own_ok = owner && otx < gw && oty < gh;
        const int sidx = oty * gw + otx;
        const float usx = (float)(S * otx) + half, usy = (float)(S * oty) + half;
        const float rsx = (usx - cxk) / fxk, rsy = (usy - cyk) / fyk;   // r_s (z = 1)
        float id = 0.f, nx = 0.f, ny = 0.f, nz = -1.f;
        uint32_t flags = 0u;
        if (own_ok) {
            id = ((gptr<float>)Kd->inv_depth)[sidx];
            nx = ((gptr<float>)Kd->nx)[sidx];
            ny = ((gptr<float>)Kd->ny)[sidx];
            nz = ((gptr<float>)Kd->nz)[sidx];
            flags = ((gptr<uint32_t>)Kd->flags)[sidx] & ~F_GN_BITS;
        }
        bool alive = own_ok;
        bool updated = false;
        float cost_out = 0.f;
        int nv_out = 0;
        float lam = lm0;             // Levenberg-Marquardt damping of this surfel
        float b1x = 0.f, b1y = 0.f, b1z = 0.f, b2x = 0.f, b2y = 0.f, b2z = 0.f;
        // r_s is the item's: written once (the words are the previous item's
        // until the sync before the pair words, which is behind us)
        if (owner) {
            float* o = lst + own * ST_WORDS;
            o[ST_RSX] = rsx; o[ST_RSY] = rsy;
        }

        for (int it = 0; it < iters; ++it) {
            const bool last = (it == iters - 1);
            // the cost is summed on the last iteration and for the damped
            // variant: a wave-uniform flag, kept in a scalar register
            const bool with_cost = __builtin_amdgcn_readfirstlane((int)(last || lm)) != 0;
            // ---- owners: degeneracy, tangent basis, broadcast of the state
            if (owner) {
                const float* os = lst + own * ST_WORDS;
                const float c = nx * os[ST_RSX] + ny * os[ST_RSY] + nz;     // n . r_s
                if (alive && fabsf(c) < 1e-6f) {
                    flags |= F_DEGENERATE;
                    alive = false;
                    cost_out = 0.f;
                    nv_out = 0;
                }
                tangent_basis(nx, ny, nz, b1x, b1y, b1z, b2x, b2y, b2z);
                float* o = lst + own * ST_WORDS;
                o[ST_ID] = id; o[ST_NX] = nx; o[ST_NY] = ny; o[ST_NZ] = nz;
                o[ST_B1X] = b1x; o[ST_B1Y] = b1y; o[ST_B1Z] = b1z;
                o[ST_B2X] = b2x; o[ST_B2Y] = b2y; o[ST_B2Z] = b2z;
                o[ST_INVC] = rcp_fast(c);                    // |c| >= 1e-6 where used
                o[ST_ALIVE] = alive ? 1.f : 0.f;
                o[ST_FLAGS] = __uint_as_float(flags); o[ST_LAM] = lam;
                o[ST_COSTO] = cost_out; o[ST_NVO] = __int_as_float(nv_out);
            }
            wave_sync();
            // ---- pixel lanes: linearise every group and reduce per surfel
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const float* st = lst + (k * SLOTS + r) * ST_WORDS;
                const float4 sa = *(const float4*)(st + 0);      // id, nx, ny, nz
                const float sid = sa.x, snx = sa.y, sny = sa.z;
                const float inv_c = st[ST_INVC];
                const bool salive = st[ST_ALIVE] != 0.f;
                const int tx = it0x + (k % G.gx) * TX + r % TX, ty = it0y + (k / G.gx) * TY + r / TX;
                // this lane's share of J^T W J = sum_u A_u g g^T and
                // J^T W r = sum_u B_u g (the frame sum hoisted), its valid
                // count and cost, over its pixels in order
                float ph[9], pnv, pcs;
                // frame-independent per-pixel terms (Eq. 3, Eq. 9)
                bool pix_ok[PPL];
                // sigma_u = n . (r_u - r_s) / (n . r_s): the lane's first
                // pixel's, and the step between its pixels (same column);
                // id_u = id_s (1 + sigma_u) steps by id_s dsig
                const float cnx = snx * inv_c, cny = sny * inv_c;
                const float sig0 = fmaf(cny, dry0, cnx * drx0);
                const float dsig = cny * dyr_f;
                const float idu0 = fmaf(sid, sig0, sid);
                const float didu = sid * dsig;
#pragma unroll
                for (int j = 0; j < PPL; ++j) {
                    const float sig = j == 0 ? sig0 : fmaf((float)j, dsig, sig0);
                    pix_ok[j] = salive && (fmaf(sid, sig, sid) > 0.f);
                }
                // the first pixel's offset from the anchor block centre; the
                // lane's later pixels lie DYR rows apart in the same column
                const float bdx = (float)(S * tx + pxs[0] - bpx) - 0.5f * (float)(G.ab * S - 1);
                const float bdy = (float)(S * ty + pys[0] - bpy) - 0.5f * (float)(G.ab * S - 1);
                float A[PPL], B[PPL], cst[PPL];
                unsigned nvp = 0u;
#pragma unroll
                for (int j = 0; j < PPL; ++j) {
                    A[j] = 0.f; B[j] = 0.f; cst[j] = 0.f;
                }
                if (with_cost)
                    frame_loop_px<T, true, PPL, BY_ROW>(pairs, fr, nf, bdx, bdy, DYR, idu0, didu, pix_ok, pitch_b,
                                                img_bytes, wm1, hm1, ikf[k], hk, img_scale, A, B, cst, nvp);
                else
                    frame_loop_px<T, false, PPL, BY_ROW>(pairs, fr, nf, bdx, bdy, DYR, idu0, didu, pix_ok, pitch_b,
                                                 img_bytes, wm1, hm1, ikf[k], hk, img_scale, A, B, cst, nvp);
                // the surfel's state and tangent basis, read again from LDS
                // after the frame loop rather than held in registers through it
                __asm__ volatile("" ::: "memory");
                const float4 sa2 = *(const float4*)(st + 0);     // id, nx, ny, nz
                const float4 sb = *(const float4*)(st + 4);      // b1, b2x
                const float4 sc = *(const float4*)(st + 8);      // b2y, b2z, 1/c, rsx
                const float srsy = st[ST_RSY];
                const float sb1x = sb.x, sb1y = sb.y, sb1z = sb.z;
                const float sb2x = sb.w, sb2y = sc.x, sb2z = sc.y, srsx = sc.w;
                const float pinv_c = sc.z;
                // g_u = (1 + sigma_u, kk b1 . d_u, kk b2 . d_u) with
                // d_u = (r_u - r_s) - sigma_u (r_s, 1) and kk = id_s / (n . r_s):
                // b . d_u = (b_x drx + b_y dry_u) - sigma_u (b . (r_s, 1)).  All
                // three are affine in the pixel's row, so each is its value at
                // the lane's first pixel plus j steps.  The depth-only ablation
                // zeroes kk, and with it the normal columns.
                const float pcnx = sa2.y * pinv_c, pcny = sa2.z * pinv_c;
                const float psig0 = fmaf(pcny, dry0, pcnx * drx0);
                const float pdsig = pcny * dyr_f;
                const float kk = depth_only ? 0.f : sa2.x * pinv_c;
                const float k1x = kk * sb1x, k1y = kk * sb1y, k2x = kk * sb2x, k2y = kk * sb2y;
                const float q1 = kk * fmaf(sb1x, srsx, fmaf(sb1y, srsy, sb1z));
                const float q2 = kk * fmaf(sb2x, srsx, fmaf(sb2y, srsy, sb2z));
                const float g00 = 1.f + psig0;
                const float g10 = fmaf(-psig0, q1, fmaf(k1y, dry0, k1x * drx0));
                const float g20 = fmaf(-psig0, q2, fmaf(k2y, dry0, k2x * drx0));
                const float dg1 = fmaf(-pdsig, q1, k1y * dyr_f);
                const float dg2 = fmaf(-pdsig, q2, k2y * dyr_f);
                if constexpr (PPL == 4) {
                    // sum_j A_j g_j g_j^T and sum_j B_j g_j with g_j = ga + j gb,
                    // through the lane's moments S_m = sum_j j^m A_j and
                    // T_m = sum_j j^m B_j: with u = S0 ga + S1 gb and
                    // v = S1 ga + S2 gb, H = u ga^T + v gb^T and b = T0 ga + T1 gb
                    // (42 instructions for the four pixels against 60 per pixel)
                    const float S0 = (A[0] + A[1]) + (A[2] + A[3]);
                    const float S1 = fmaf(3.f, A[3], fmaf(2.f, A[2], A[1]));
                    const float S2 = fmaf(9.f, A[3], fmaf(4.f, A[2], A[1]));
                    const float T0 = (B[0] + B[1]) + (B[2] + B[3]);
                    const float T1 = fmaf(3.f, B[3], fmaf(2.f, B[2], B[1]));
                    const float ga[3] = {g00, g10, g20}, gb[3] = {pdsig, dg1, dg2};
                    float uu[3], vv[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        uu[a] = fmaf(S1, gb[a], S0 * ga[a]);
                        vv[a] = fmaf(S2, gb[a], S1 * ga[a]);
                    }
                    ph[0] = fmaf(vv[0], gb[0], uu[0] * ga[0]);     // H00
                    ph[1] = fmaf(vv[0], gb[1], uu[0] * ga[1]);     // H01
                    ph[2] = fmaf(vv[0], gb[2], uu[0] * ga[2]);     // H02
                    ph[3] = fmaf(vv[1], gb[1], uu[1] * ga[1]);     // H11
                    ph[4] = fmaf(vv[1], gb[2], uu[1] * ga[2]);     // H12
                    ph[5] = fmaf(vv[2], gb[2], uu[2] * ga[2]);     // H22
#pragma unroll
                    for (int a = 0; a < 3; ++a) ph[6 + a] = fmaf(T1, gb[a], T0 * ga[a]);
                    pcs = (cst[0] + cst[1]) + (cst[2] + cst[3]);
                } else {
#pragma unroll
                    for (int j = 0; j < PPL; ++j) {
                        const float g0 = fmaf((float)j, pdsig, g00);
                        const float g1 = fmaf((float)j, dg1, g10);
                        const float g2 = fmaf((float)j, dg2, g20);
                        const float ag0 = A[j] * g0, ag1 = A[j] * g1, ag2 = A[j] * g2;
                        const float u[9] = {ag0, ag0, ag0, ag1, ag1, ag2, B[j], B[j], B[j]};
                        const float v[9] = {g0, g1, g2, g1, g2, g2, g0, g1, g2};
#pragma unroll
                        for (int e = 0; e < 9; ++e) ph[e] = (j == 0) ? u[e] * v[e] : fmaf(u[e], v[e], ph[e]);
                        pcs = (j == 0) ? cst[j] : pcs + cst[j];
                    }
                }
                // the lane's valid samples: the byte counters summed (v_sad_u8)
                pnv = (float)__builtin_amdgcn_sad_u8(nvp, 0u, 0u);
                // reduced two at a time: lane 0 of the surfel ends with words
                // 0, 2, 4, 6, 8 and lane 1 with words 1, 3, 5, 7, 9 (the valid
                // count as an exact float)
                float s0, s1, s2, s3, s4;
                {
                    // No FMA contraction: each butterfly step must be a plain
                    // add of two rounded values so that the sums do not depend
                    // on which lane forms them.
#pragma clang fp contract(off)
                    const bool odd = (p & 1) != 0;
                    s0 = pair_sum<LANES>(ph[0], ph[1], odd);     // H00 | H01
                    s1 = pair_sum<LANES>(ph[2], ph[3], odd);     // H02 | H11
                    s2 = pair_sum<LANES>(ph[4], ph[5], odd);     // H12 | H22
                    s3 = pair_sum<LANES>(ph[6], ph[7], odd);     // b0  | b1
                    s4 = pair_sum<LANES>(ph[8], pnv, odd);       // b2  | nv
                }
                // In a 4-lane surfel lanes 2 and 3 end with the sums of lanes 0
                // and 1, formed from the same two partial sums (the adds
                // commute), so they store the same words: no branch, and the
                // last butterfly add stays a DPP add over the whole wavefront.
                float* const o = lsm + (k * SLOTS + r) * SM_WORDS;
                if (LANES == 4 || p < 2) {
                    const int w = p & 1;
                    o[w] = s0; o[w + 2] = s1; o[w + 4] = s2; o[w + 6] = s3; o[w + 8] = s4;
                }
                if (with_cost) {
                    const float cs = group_sum<LANES>(pcs);    // 4 lanes: the same in each
                    if (LANES == 4 || p == 0) o[SM_COST] = cs;
                }
            }
            wave_sync();
            // the owner's state and tangent basis, read back from the words it
            // wrote before the group loop rather than held in registers
            // through the frame loops
            __asm__ volatile("" ::: "memory");
            if (owner) {
                const float* o = lst + own * ST_WORDS;
                const float4 w0 = *(const float4*)(o + 0);
                const float4 w1 = *(const float4*)(o + 4);
                const float4 w2 = *(const float4*)(o + 8);
                const float4 w3 = *(const float4*)(o + 12);
                const float4 w4 = *(const float4*)(o + 16);
                id = w0.x; nx = w0.y; ny = w0.z; nz = w0.w;
                b1x = w1.x; b1y = w1.y; b1z = w1.z; b2x = w1.w; b2y = w2.x; b2z = w2.y;
                alive = w3.y != 0.f;
                flags = __float_as_uint(w3.z); lam = w3.w;
                cost_out = w4.x; nv_out = __float_as_int(w4.y);
            }
            // ---- owners: solve, update (Levenberg-Marquardt candidate test below)
            bool cand = false;
            float id_c = 0.f, nx_c = 0.f, ny_c = 0.f, nz_c = 0.f, cost_here = 0.f;
            int nv = 0;
            if (owner) {
                // The step of owner_step, written out here: as a call (forced
                // inline) the compiler allocates 5-10 more VGPRs for this
                // kernel, which spills in the default plan and costs the
                // one-group plans their sixth wavefront per SIMD.  The text
                // between the markers must equal owner_step's body; a CPU test
                // compares the two.  kappa^2 is formed here, each iteration,
                // rather than held in a register through the frame loops.
                float kappa_it = kappa_s;
                __asm__ volatile("" : "+s"(kappa_it));
                const float kap2 = kappa_it * kappa_it;
                // owner_step body begin
                const float* sm = lsm + own * SM_WORDS;
                const float H00 = sm[SM_H00], H01 = sm[SM_H01], H02 = sm[SM_H02];
                const float H11 = sm[SM_H11], H12 = sm[SM_H12], H22 = sm[SM_H22];
                const float bb0 = sm[SM_B0], bb1 = sm[SM_B1], bb2 = sm[SM_B2];
                nv = (int)sm[SM_NV];
                cost_here = sm[SM_COST];
                if (alive && last) cost_out = cost_here;
                if (alive) {
                    nv_out = nv;
                    float d0s = 0.f, d1s = 0.f, d2s = 0.f;
                    bool ok = true;
                    if (nv < 3) {
                        flags |= F_FEW_SAMPLES;
                        ok = false;
                    }
                    const float dd = 1.f + lam;          // (H + lam diag H): equilibrated diagonal
                    if (ok && depth_only) {
                        if (H00 > 0.f && isfinite(H00)) {
                            d0s = -bb0 * rcp_fast(H00 * dd);
                        } else {
                            flags |= F_SOLVE_FAIL;
                            ok = false;
                        }
                    } else if (ok) {
                        // equilibrate: E = D^-1/2 H D^-1/2 (unit diagonal).  The float
                        // solve is formed unconditionally (no branches: the tests below
                        // are combined with |) and replaced by the double-precision one
                        // where a diagonal is not positive and finite or the system is
                        // too ill-conditioned for float.
                        const float maxd = fmaxf(H00, fmaxf(H11, H22));
                        const float e0 = __frsqrt_rn(H00), e1 = __frsqrt_rn(H11), e2 = __frsqrt_rn(H22);
                        const float e01 = H01 * e0 * e1, e02 = H02 * e0 * e2, e12 = H12 * e1 * e2;
                        // adjugate and determinant of E (diagonal dd = 1 + lambda)
                        const float d2 = dd * dd;
                        const float c00 = fmaf(-e12, e12, d2), c11 = fmaf(-e02, e02, d2);
                        const float c22 = fmaf(-e01, e01, d2);
                        const float c01 = fmaf(e02, e12, -dd * e01), c02 = fmaf(e01, e12, -dd * e02);
                        const float c12 = fmaf(e01, e02, -dd * e12);
                        const float det = fmaf(e01, c01, fmaf(e02, c02, dd * c00));
                        // kappa_F(E)^2 = ||E||_F^2 ||adj E||_F^2 / det^2  (>= kappa_2(E)^2)
                        const float fro2 = 3.f * d2 + 2.f * (e01 * e01 + e02 * e02 + e12 * e12);
                        const float adj2 = c00 * c00 + c11 * c11 + c22 * c22 +
                                           2.f * (c01 * c01 + c02 * c02 + c12 * c12);
                        // raw Cholesky pivots are H_jj times the equilibrated ones
                        const float p1 = c22 * rcp_fast(dd);   // dd - e01^2 / dd (only compared)
                        const float p2 = det * rcp_fast(c22);  // (only compared)
                        const bool need64 = !(H00 > 0.f) | !(H11 > 0.f) | !(H22 > 0.f) | !isfinite(maxd) |
                                            !(fro2 * adj2 <= kap2 * det * det) | !(det > 0.f) | !(c22 > 0.f) |
                                            !(H11 * p1 > 1e-10f * maxd * dd) | !(H22 * p2 > 1e-10f * maxd * dd);
                        {
                            const float bh0 = bb0 * e0, bh1 = bb1 * e1, bh2 = bb2 * e2;
                            const float idet = rcp_fast(det);
                            d0s = -(c00 * bh0 + c01 * bh1 + c02 * bh2) * idet * e0;
                            d1s = -(c01 * bh0 + c11 * bh1 + c12 * bh2) * idet * e1;
                            d2s = -(c02 * bh0 + c12 * bh1 + c22 * bh2) * idet * e2;
                        }
                        if (need64) {
                            flags |= F_FP64_SOLVE;
                            double dd0 = 0.0, dd1 = 0.0, dd2 = 0.0;
                            const double dmp = 1.0 + (double)lam;
                            if (solve3_fp64((double)H00 * dmp, H01, H02, (double)H11 * dmp, H12,
                                            (double)H22 * dmp, bb0, bb1, bb2, dd0, dd1, dd2)) {
                                d0s = (float)dd0; d1s = (float)dd1; d2s = (float)dd2;
                            } else {
                                flags |= F_SOLVE_FAIL;
                                ok = false;
                            }
                        }
                    }
                    if (ok) {
                        // update: id_s += d0; n = normalise(n + d1 b1 + d2 b2) (the
                        // depth-only ablation moves id_s alone and keeps n)
                        id_c = id + d0s;
                        nx_c = nx; ny_c = ny; nz_c = nz;
                        bool ok_step;
                        if (depth_only) {
                            ok_step = (id_c > 0.f) && isfinite(id_c);
                        } else {
                            const float mx = fmaf(d1s, b1x, fmaf(d2s, b2x, nx));
                            const float my = fmaf(d1s, b1y, fmaf(d2s, b2y, ny));
                            const float mz = fmaf(d1s, b1z, fmaf(d2s, b2z, nz));
                            const float l2 = mx * mx + my * my + mz * mz;
                            ok_step = (id_c > 0.f) && isfinite(id_c) && (l2 > 0.f) && isfinite(l2);
                            if (ok_step) {
                                const float il = __frsqrt_rn(l2);
                                nx_c = mx * il; ny_c = my * il; nz_c = mz * il;
                            }
                        }
                        if (!ok_step) {
                            flags |= F_REJECTED;
                            if (lm) lam *= 10.f;
                        } else {
                            cand = true;
                        }
                    }
                }
                // owner_step body end
            }
            if (lm) {
                // Levenberg-Marquardt: the candidate's cost over the pixels,
                // then the acceptance test (lm_accept)
                float inv_cc = 0.f;
                bool cand_ok = cand;
                if (owner && cand) {
                    const float cc = nx_c * rsx + ny_c * rsy + nz_c;
                    if (fabsf(cc) < 1e-6f) {             // candidate plane contains r_s
                        flags |= F_REJECTED;
                        lam *= 10.f;
                        cand_ok = false;
                    }
                    inv_cc = rcp_fast(cc);
                }
                if (owner) {
                    float* o = lst + own * ST_WORDS;
                    o[ST_ID] = id_c; o[ST_NX] = nx_c; o[ST_NY] = ny_c; o[ST_NZ] = nz_c;
                    o[ST_INVC] = inv_cc;
                    o[ST_ALIVE] = cand_ok ? 1.f : 0.f;
                }
                wave_sync();
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const float* st = lst + (k * SLOTS + r) * ST_WORDS;
                    const float4 sa = *(const float4*)(st + 0);
                    const float inv_c = st[ST_INVC];
                    const bool calive = st[ST_ALIVE] != 0.f;
                    const int tx = it0x + (k % G.gx) * TX + r % TX, ty = it0y + (k / G.gx) * TY + r / TX;
                    float cst2 = 0.f;
                    int nv2l = 0;
                    const float cnx = sa.y * inv_c, cny = sa.z * inv_c;
                    const float sig0 = fmaf(cny, dry0, cnx * drx0);
                    const float dsig = cny * dyr_f;
#pragma unroll
                    for (int j = 0; j < PPL; ++j) {
                        const float sig = j == 0 ? sig0 : fmaf((float)j, dsig, sig0);
                        const float idu_c = fmaf(sa.x, sig, sa.x);
                        float bdx = (float)(S * tx + pxs[j] - bpx) - 0.5f * (float)(G.ab * S - 1);
                        float bdy = (float)(S * ty + pys[j] - bpy) - 0.5f * (float)(G.ab * S - 1);
                        // formed here, not kept from the item's start through the
                        // iterations (registers)
                        __asm__ volatile("" : "+v"(bdx), "+v"(bdy));
                        frame_cost<T, BY_ROW>(pairs, fr, nf, bdx, bdy, idu_c, calive && (idu_c > 0.f), pitch_b,
                                      img_bytes, wm1, hm1, ikf[k][j], hk, img_scale, cst2, nv2l);
                    }
                    const float c2 = group_sum<LANES>(cst2);
                    const int n2 = group_sum<LANES>(nv2l);
                    if (p == 0) {
                        float* o = lsm + (k * SLOTS + r) * SM_WORDS;
                        o[SM_COST] = c2;
                        o[SM_NV] = __int_as_float(n2);
                    }
                }
                wave_sync();
                if (owner && cand_ok) {
                    const float* sm = lsm + own * SM_WORDS;
                    cand_ok = lm_accept(sm[SM_COST], __float_as_int(sm[SM_NV]), cost_here, nv, lam);
                }
                cand = cand_ok;
            }
            if (owner && cand) {
                id = id_c;
                nx = nx_c; ny = ny_c; nz = nz_c;
                updated = true;
            }
        }
        if (own_ok) {
            ((gmut<float>)Kd->inv_depth)[sidx] = id;
            ((gmut<float>)Kd->nx)[sidx] = nx;
            ((gmut<float>)Kd->ny)[sidx] = ny;
            ((gmut<float>)Kd->nz)[sidx] = nz;
            ((gmut<uint32_t>)Kd->flags)[sidx] = flags;
            ((gmut<float>)Kd->cost)[sidx] = iters > 0 ? cost_out : 0.f;
            ((gmut<uint32_t>)Kd->nvalid)[sidx] = (uint32_t)(iters > 0 ? nv_out : 0);
            if (updated) ((gmut<uint32_t>)Kd->last_update)[sidx] = stamp;
        }
    }
}

// ----------------------------------------------------------- render kernel --

// Inverse Depth Calculation section: each pixel takes Eq. 3 of its surfel,
// id_u = id_s (1 + sigma), sigma = n . (r_u - r_s) / (n . r_s).  A thread
// renders one segment: the up-to-S pixels of one image row that lie in one
// tile column (segments past the grid write "no measurement"), so a surfel's
// state is read once per segment.  Segments are numbered keyframe after
// keyframe (only keyframes with an output).  A block takes runs of 256
// consecutive segments: its first thread finds the run's keyframe, and only
// threads whose segment lies past that keyframe search for their own.

// The keyframe owning segment g: the last one whose base is <= g (keyframes
// without an output add no segments, so the next base is larger than g only
// past the owner).
__device__ __forceinline__ int render_owner(cptr<KfDev> kfs, int n_kf, int64_t g) {
    int lo = 0, hi = n_kf - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (kfs[mid].pixel_base <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(256) void render_kernel(const BatchHeader* __restrict__ hdr_) {
    const cptr<BatchHeader> hdr = (cptr<BatchHeader>)hdr_;
    const cptr<KfDev> kfs = (cptr<KfDev>)hdr->kfs;
    const int n_kf = hdr->n_kf;
    const int64_t total = hdr->total_pixels;           // render segments
    __shared__ int s_kf;
    // the loop bounds are the same for every thread of a block
    for (int64_t g0 = (int64_t)blockIdx.x * blockDim.x; g0 < total; g0 += (int64_t)gridDim.x * blockDim.x) {
        __syncthreads();                                // the previous run's s_kf is read
        if (threadIdx.x == 0) s_kf = render_owner(kfs, n_kf, g0);
        __syncthreads();
        const int64_t g = g0 + threadIdx.x;
        if (g >= total) continue;
        int kidx = s_kf;
        {
            const cptr<KfDev> kh = kfs + kidx;
            const int64_t nseg = (int64_t)kh->height * ((kh->width + kh->patch - 1) / kh->patch);
            if (!(kh->inv_depth_out && g >= kh->pixel_base && g < kh->pixel_base + nseg))
                kidx = render_owner(kfs, n_kf, g);
        }
        const cptr<KfDev> K = kfs + kidx;
        const int W = K->width, S = K->patch;
        const int nsx = (W + S - 1) / S;
        const int sg = (int)(g - K->pixel_base);
        const int y = sg / nsx, tx = sg - y * nsx;
        const int x0 = tx * S, ty = y >> __builtin_ctz(S);    // S is 4, 8 or 16
        const float half = 0.5f * (float)(S - 1);
        float* const out = K->inv_depth_out + (size_t)y * W + x0;
        int32_t* const idx_out = K->index_out ? K->index_out + (size_t)y * W + x0 : nullptr;
        bool ok = false;
        int i = -1;
        // three divisions per segment; the pixels multiply by the reciprocals
        const float ifx = 1.f / K->fx, ify = 1.f / K->fy;
        float id = 0.f, nx = 0.f, ny = 0.f, inv_c = 1.f, usx = 0.f, usy = 0.f;
        if (tx < K->gw && ty < K->gh) {
            i = ty * K->gw + tx;
            // the state is loaded with the flags (one round trip, not two);
            // a flagged surfel's values are not used
            const uint32_t fl = K->flags[i];
            const float snx = K->nx[i], sny = K->ny[i], snz = K->nz[i], sid = K->inv_depth[i];
            // (kept in front of the flag test, where the compiler would sink them)
            __asm__ volatile("" ::"v"(snx), "v"(sny), "v"(snz), "v"(sid));
            if (!(fl & (F_DEGENERATE | F_UNINIT))) {
                usx = (float)(S * tx) + half;
                usy = (float)(S * ty) + half;
                const float rsx = (usx - K->cx) * ifx, rsy = (usy - K->cy) * ify;
                nx = snx;
                ny = sny;
                const float c = nx * rsx + ny * rsy + snz;
                id = sid;
                ok = fabsf(c) >= 1e-6f;
                inv_c = 1.f / c;
            }
        }
        const float dry = ((float)y - usy) * ify;
        const int n_px = min(S, W - x0);
        // Eq. 3 at pixel x0 + j of the segment
        auto pixel = [&](int j, float& val, int& who) {
            val = 0.f;
            who = -1;
            if (ok) {
                const float drx = ((float)(x0 + j) - usx) * ifx;
                const float sigma = (nx * drx + ny * dry) * inv_c;
                const float idu = fmaf(id, sigma, id);
                if (idu > 0.f && isfinite(idu)) {
                    val = idu;
                    who = i;
                }
            }
        };
        if (S == 4) {
            float v[4];
            int w[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) pixel(j, v[j], w[j]);
            // a whole 16-byte aligned segment in one store, else pixel by pixel
            if (n_px == 4 && ((uintptr_t)out & 15u) == 0) {
                *(float4*)out = make_float4(v[0], v[1], v[2], v[3]);
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (j < n_px) out[j] = v[j];
            }
            if (idx_out) {
                if (n_px == 4 && ((uintptr_t)idx_out & 15u) == 0) {
                    *(int4*)idx_out = make_int4(w[0], w[1], w[2], w[3]);
                } else {
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (j < n_px) idx_out[j] = w[j];
                }
            }
        } else {
            for (int j = 0; j < n_px; ++j) {
                float v;
                int w;
                pixel(j, v, w);
                out[j] = v;
                if (idx_out) idx_out[j] = w;
            }
        }
    }
}

// ----------------------------------------------------------- regrid kernels --

// Surfel reference-frame change (Eq. 10) and re-gridding into the tiles of
// another keyframe.  Every landing decision (destination tile, closest
// surfel) is taken in double with a fixed operation order and no
// contraction, so it is the same decision the plain double definition takes.
struct Land {
    double idp, rp0, rp1, np0, np1, np2;
    int tile;
};

__device__ __forceinline__ bool regrid_land(const RegridArgs& a, int i, Land& L) {
#pragma clang fp contract(off)
    const int S0 = a.src_patch, gw0 = a.src_w / S0;
    if (a.src.flags[i] & (F_DEGENERATE | F_UNINIT)) return false;
    const double id = (double)a.src.inv_depth[i];
    if (!(id > 0.0) || !isfinite(id)) return false;
    const double usx = S0 * (i % gw0) + 0.5 * (S0 - 1), usy = S0 * (i / gw0) + 0.5 * (S0 - 1);
    const double rs0 = (usx - a.src_K[2]) / a.src_K[0], rs1 = (usy - a.src_K[3]) / a.src_K[1];
    const double p00 = rs0 / id, p01 = rs1 / id, p02 = 1.0 / id;          // Eq. 1
    const double n0 = a.src.nx[i], n1 = a.src.ny[i], n2 = a.src.nz[i];
    const double* R = a.R;
    const double p10 = R[0] * p00 + R[1] * p01 + R[2] * p02 + a.t[0];
    const double p11 = R[3] * p00 + R[4] * p01 + R[5] * p02 + a.t[1];
    const double p12 = R[6] * p00 + R[7] * p01 + R[8] * p02 + a.t[2];
    L.np0 = R[0] * n0 + R[1] * n1 + R[2] * n2;
    L.np1 = R[3] * n0 + R[4] * n1 + R[5] * n2;
    L.np2 = R[6] * n0 + R[7] * n1 + R[8] * n2;
    if (!(p12 > 0.0)) return false;
    L.rp0 = p10 / p12;
    L.rp1 = p11 / p12;
    const double ux = a.dst_K[0] * L.rp0 + a.dst_K[2], uy = a.dst_K[1] * L.rp1 + a.dst_K[3];
    const double px = floor(ux + 0.5), py = floor(uy + 0.5);          // nearest pixel
    const int S1 = a.dst_patch, gw1 = a.dst_w / S1, gh1 = a.dst_h / S1;
    if (!(px >= 0.0 && px < (double)(gw1 * S1) && py >= 0.0 && py < (double)(gh1 * S1))) return false;
    L.tile = ((int)py / S1) * gw1 + (int)px / S1;
    L.idp = 1.0 / p12;
    return true;
}

// The re-gridding kernels run over a table of keyframe pairs in wavefronts
// of 64 lanes that never span two pairs: pair k's sources (destination
// tiles) take the wavefronts from src_wave (dst_wave) on, so the entry is
// the last whose first wavefront is <= the wavefront's number.  It is found
// and read with wavefront-uniform (scalar) loads.
template <bool DST>
__device__ __forceinline__ int regrid_entry_of_wave(const RegridArgs* __restrict__ tab, int n, int wv) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((DST ? tab[mid].dst_wave : tab[mid].src_wave) <= wv) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// The wavefront's number among the grid's (four wavefronts per workgroup),
// uniform for the compiler, and the grid's count of wavefronts.
__device__ __forceinline__ int grid_wave() {
    return __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
}
__device__ __forceinline__ int grid_waves() { return (int)gridDim.x * 4; }

__global__ __launch_bounds__(256) void regrid_clear_kernel(const RegridArgs* __restrict__ tab, int n_pairs,
                                                           int dst_waves) {
    const int lane = threadIdx.x & 63;
    for (int wv = grid_wave(); wv < dst_waves; wv += grid_waves()) {
        const RegridArgs& a = tab[regrid_entry_of_wave<true>(tab, n_pairs, wv)];
        const int j = (wv - a.dst_wave) * 64 + lane;
        if (j < a.dst_count) {
            a.best[j] = 0ull;
            a.win[j] = 0x7fffffff;
        }
    }
}

// pass 0: closest landing per tile (1/p'_z > 0, so its bits order like the
// value); pass 1: the lowest source index among the closest
__global__ __launch_bounds__(256) void regrid_scatter_kernel(const RegridArgs* __restrict__ tab, int n_pairs,
                                                             int src_waves, int pass) {
    const int lane = threadIdx.x & 63;
    for (int wv = grid_wave(); wv < src_waves; wv += grid_waves()) {
        const RegridArgs& a = tab[regrid_entry_of_wave<false>(tab, n_pairs, wv)];
        const int i = (wv - a.src_wave) * 64 + lane;
        Land L;
        if (i >= a.src_count || !regrid_land(a, i, L)) continue;
        const unsigned long long bits = (unsigned long long)__double_as_longlong(L.idp);
        if (pass == 0)
            atomicMax(&a.best[L.tile], bits);
        else if (a.best[L.tile] == bits)
            atomicMin(&a.win[L.tile], i);
    }
}

__global__ __launch_bounds__(256) void regrid_gather_kernel(const RegridArgs* __restrict__ tab, int n_pairs,
                                                            int dst_waves) {
#pragma clang fp contract(off)
    const int lane = threadIdx.x & 63;
    for (int wv = grid_wave(); wv < dst_waves; wv += grid_waves()) {
        const RegridArgs& a = tab[regrid_entry_of_wave<true>(tab, n_pairs, wv)];
        const int j = (wv - a.dst_wave) * 64 + lane;
        if (j >= a.dst_count) continue;
        const int S1 = a.dst_patch, gw1 = a.dst_w / S1;
        const int w = a.win[j];
        bool ok = false;
        double idt = 0.0, t0 = 0.0, t1 = 0.0, t2 = -1.0;
        Land L;
        if (w != 0x7fffffff && regrid_land(a, w, L)) {
            const double rt0 = (S1 * (j % gw1) + 0.5 * (S1 - 1) - a.dst_K[2]) / a.dst_K[0];
            const double rt1 = (S1 * (j / gw1) + 0.5 * (S1 - 1) - a.dst_K[3]) / a.dst_K[1];
            const double c1 = L.np0 * L.rp0 + L.np1 * L.rp1 + L.np2 * 1.0;
            const double ct = L.np0 * rt0 + L.np1 * rt1 + L.np2 * 1.0;
            if (fabs(c1) >= 1e-6 && fabs(ct) >= 1e-6) {
                idt = L.idp * ct / c1;                    // Eq. 3 of the moved plane at r_t
                const double l = sqrt(L.np0 * L.np0 + L.np1 * L.np1 + L.np2 * L.np2);
                if (idt > 0.0 && isfinite(idt) && l > 0.0 && isfinite(l)) {
                    t0 = L.np0 / l; t1 = L.np1 / l; t2 = L.np2 / l;
                    ok = true;
                }
            }
        }
        a.dst.inv_depth[j] = ok ? (float)idt : 0.f;
        a.dst.nx[j] = ok ? (float)t0 : 0.f;
        a.dst.ny[j] = ok ? (float)t1 : 0.f;
        a.dst.nz[j] = ok ? (float)t2 : -1.f;
        a.dst.flags[j] = ok ? 0u : F_UNINIT;
        a.dst.cost[j] = 0.f;
        a.dst.nvalid[j] = 0u;
        a.dst.last_update[j] = ok ? a.src.last_update[w] : 0u;
        a.is_new[j] = ok ? 0 : 1;
        if (a.src_index) a.src_index[j] = ok ? w : -1;
    }
}

hipError_t launch_regrid(const RegridArgs* table, int n_pairs, int src_waves, int dst_waves,
                         hipStream_t s) {
    // four wavefronts per workgroup
    auto blocks = [](int waves) { return std::max(1, std::min(65536, (waves + 3) / 4)); };
    hipLaunchKernelGGL(regrid_clear_kernel, dim3(blocks(dst_waves)), dim3(256), 0, s, table, n_pairs,
                       dst_waves);
    if (src_waves > 0) {
        hipLaunchKernelGGL(regrid_scatter_kernel, dim3(blocks(src_waves)), dim3(256), 0, s, table, n_pairs,
                           src_waves, 0);
        hipLaunchKernelGGL(regrid_scatter_kernel, dim3(blocks(src_waves)), dim3(256), 0, s, table, n_pairs,
                           src_waves, 1);
    }
    hipLaunchKernelGGL(regrid_gather_kernel, dim3(blocks(dst_waves)), dim3(256), 0, s, table, n_pairs,
                       dst_waves);
    return hipGetLastError();
}

// --------------------------------------------------------- quantize kernel --

__global__ void quantize_kernel(const float* __restrict__ src, int src_pitch, void* __restrict__ dst,
                                int dst_pitch, int width, int height, int dtype, float scale) {
    const int64_t total = (int64_t)width * height;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(g % width), y = (int)(g / width);
        const float v = src[(size_t)y * src_pitch + x];
        if (dtype == 1) {
            ((_Float16*)dst)[(size_t)y * dst_pitch + x] = (_Float16)(v / scale);
        } else {
            float c = rintf(v / scale);
            c = fminf(fmaxf(c, 0.f), 255.f);
            ((uint8_t*)dst)[(size_t)y * dst_pitch + x] = (uint8_t)c;
        }
    }
}

// ---------------------------------------------------------- static scratch --
//
// Scratch of the allocation-free entry point (sgn_transfer_surfels_static): a
// file-scope device array, one copy per GPU, held until the process ends.
// Host code never uses the name `scratch` as an address: static_scratch_on
// looks up each device's copy once, with that device current, and the
// callers pass the looked-up pointer to kernels.
static __device__ __align__(256) unsigned char scratch[SGN_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch_on(int device, void** out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

// ---------------------------------------------------------------- launchers --

hipError_t launch_setup(const BatchHeader* hdr, uint32_t* counters, int n_frames_cap, hipStream_t s) {
    int n = n_frames_cap > kNumCounters ? n_frames_cap : kNumCounters;
    int blocks = (n + 255) / 256;
    hipLaunchKernelGGL(setup_kernel, dim3(blocks), dim3(256), 0, s, hdr, counters);
    return hipGetLastError();
}

hipError_t launch_init(const BatchHeader* hdr, int grid, hipStream_t s) {
    hipLaunchKernelGGL(init_kernel, dim3(grid), dim3(256), 0, s, hdr);
    return hipGetLastError();
}

hipError_t launch_render(const BatchHeader* hdr, int grid, hipStream_t s) {
    hipLaunchKernelGGL(render_kernel, dim3(grid), dim3(256), 0, s, hdr);
    return hipGetLastError();
}

hipError_t launch_quantize(const float* src, int src_pitch, void* dst, int dst_pitch, int width,
                           int height, int dtype, float scale, hipStream_t s) {
    int64_t total = (int64_t)width * height;
    int blocks = (int)((total + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(quantize_kernel, dim3(blocks), dim3(256), 0, s, src, src_pitch, dst, dst_pitch,
                       width, height, dtype, scale);
    return hipGetLastError();
}

template <typename T, int S, int TX, int TY, int K, bool R>
static void* gn_ptr() {
    return (void*)&gn_kernel<T, S, TX, TY, K, R>;
}

template <typename T, int S, int TX, int TY, bool R, int KMAX = 4>
static void* gn_pick_groups(int groups) {
    if (groups == 1) return gn_ptr<T, S, TX, TY, 1, R>();
    if (groups == 2) return gn_ptr<T, S, TX, TY, 2, R>();
    if constexpr (KMAX >= 4)
        if (groups == 4) return gn_ptr<T, S, TX, TY, 4, R>();
    return nullptr;
}

template <typename T, bool R>
static void* gn_pick(const GnVariant& v) {
    if (v.patch == 8 && v.tiles_x == 1 && v.tiles_y == 1) return gn_pick_groups<T, 8, 1, 1, R>(v.groups);
    // a 16 x 16 surfel is its own anchor block: one group per item
    if (v.patch == 16 && v.tiles_x == 1 && v.tiles_y == 1 && v.groups == 1) return gn_ptr<T, 16, 1, 1, 1, R>();
    if (v.patch == 4 && v.tiles_x == 4 && v.tiles_y == 1) return gn_pick_groups<T, 4, 4, 1, R>(v.groups);
    if (v.patch == 4 && v.tiles_x == 2 && v.tiles_y == 2) return gn_pick_groups<T, 4, 2, 2, R>(v.groups);
    if (v.patch == 4 && v.tiles_x == 1 && v.tiles_y == 4) return gn_pick_groups<T, 4, 1, 4, R>(v.groups);
    // eight 4 x 4 surfels per wavefront, two pixels per lane: one or two groups
    if (v.patch == 4 && v.tiles_x == 4 && v.tiles_y == 2) return gn_pick_groups<T, 4, 4, 2, R, 2>(v.groups);
    if (v.patch == 4 && v.tiles_x == 2 && v.tiles_y == 4) return gn_pick_groups<T, 4, 2, 4, R, 2>(v.groups);
    // sixteen 4 x 4 surfels (a whole anchor block) per wavefront, four pixels per lane
    if (v.patch == 4 && v.tiles_x == 4 && v.tiles_y == 4 && v.groups == 1) return gn_ptr<T, 4, 4, 4, 1, R>();
    return nullptr;
}

static void* gn_select(const GnVariant& v) {
    if (v.lds) return nullptr;
    if (v.dtype == 0) return v.by_row ? gn_pick<float, true>(v) : gn_pick<float, false>(v);
    if (v.dtype == 1) return v.by_row ? gn_pick<_Float16, true>(v) : gn_pick<_Float16, false>(v);
    if (v.dtype == 2) return v.by_row ? gn_pick<uint8_t, true>(v) : gn_pick<uint8_t, false>(v);
    return nullptr;
}

bool gn_variant_supported(const GnVariant& v) { return gn_select(v) != nullptr; }

int gn_blocks_per_cu(const GnVariant& v) {
    void* f = gn_select(v);
    if (!f) return 0;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, kBlockThreads, 0) != hipSuccess) return 0;
    return n;
}

hipError_t launch_gn(const GnVariant& v, const BatchHeader* hdr, uint32_t* counters, int persistent,
                     int grid_blocks, hipStream_t s) {
    void* f = gn_select(v);
    if (!f) return hipErrorInvalidValue;
    void* args[] = {(void*)&hdr, (void*)&counters, (void*)&persistent};
    return hipLaunchKernel(f, dim3(grid_blocks), dim3(kBlockThreads), args, 0, s);
}

// ------------------------------------------------------------ disc surfels --
//
// Disc surfels (Eq. 4): surfel s is centred at u_s = (ux, uy) in keyframe
// pixels and covers the pixels u (inside the image) with |u - u_s| < r, r
// the same for every surfel of a keyframe (0 < r <= kDiscMaxRadius).
// Membership is decided as dx^2 + dy^2 < r^2 in double (dx = x - ux is
// exact there).  A disc's pixels are numbered row by row; a surfel held by
// LANES lanes gives lane l pixels l, l + LANES, ... (at most 512 / LANES).

constexpr int kDiscMaxRows = 2 * (int)kDiscMaxRadius + 2;
constexpr int kDiscPPL = 8;        // 512 pixels > pi (12 + sqrt(2)/2)^2, the largest disc
constexpr int kDiscRowWords = 2 * kDiscMaxRows + 2;
// largest ceil(beta r) of the neighbour search (beta <= 4, r <= 12)
constexpr int kDiscMaxWindowReach = 4 * (int)kDiscMaxRadius;

struct DiscRows {
    int y0, nrows, total;
};

// A disc pixel's slot in LDS: its offset from the anchor pixel as two int8
// (|offset| <= 12) in the low half-word and, for f16 and u8 images, the
// keyframe value's stored bits in the high half-word (f32 values go to a
// float array of their own).
template <typename T> struct DiscSlot {
    static constexpr bool packed = true;
};
template <> struct DiscSlot<float> {
    static constexpr bool packed = false;
};
__device__ __forceinline__ uint32_t slot_bits(_Float16 v) { return __builtin_bit_cast(uint16_t, v); }
__device__ __forceinline__ uint32_t slot_bits(uint8_t v) { return v; }
__device__ __forceinline__ uint32_t slot_bits(float) { return 0u; }
template <typename T>
__device__ __forceinline__ float slot_value(uint32_t pk);
template <>
__device__ __forceinline__ float slot_value<_Float16>(uint32_t pk) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(pk >> 16));
}
template <>
__device__ __forceinline__ float slot_value<uint8_t>(uint32_t pk) { return (float)(pk >> 16); }
template <>
__device__ __forceinline__ float slot_value<float>(uint32_t) { return 0.f; }

// The rows of one disc (clipped to the image): the surfel's lanes below the
// row count (hl is the lane's index among the surfel's LANES lanes) find
// their row's run of pixels (a disc meets a row in one run), and a scan over
// those lanes forms the running counts.  row_x0[i] is the first column of
// row y0 + i and row_start[i] the number of disc pixels before it.  A
// non-finite centre gives an empty disc.  Every lane passes the same
// synchronisation point; the caller synchronises the wavefront before.
template <int LANES>
__device__ DiscRows disc_rows(float ux, float uy, float radius, int W, int H, int hl, int* row_x0,
                              int* row_start) {
#pragma clang fp contract(off)
    DiscRows d{0, 0, 0};
    const double cx = (double)ux, cy = (double)uy, r = (double)radius, r2 = r * r;
    const double xlo = fmax(0.0, ceil(cx - r)), xhi = fmin((double)(W - 1), floor(cx + r));
    const double ylo = fmax(0.0, ceil(cy - r)), yhi = fmin((double)(H - 1), floor(cy + r));
    const bool ok = isfinite(cx) && isfinite(cy) && xlo <= xhi && ylo <= yhi &&
                    yhi - ylo < (double)(kDiscMaxRows - 1);
    int x0 = 0, x1 = -1;
    if (ok) {
        x0 = (int)xlo;
        x1 = (int)xhi;
        d.y0 = (int)ylo;
        d.nrows = (int)yhi - d.y0 + 1;
    }
    int first = x0, cnt = 0;
    if (hl < d.nrows) {
        const double dy = (double)(d.y0 + hl) - cy;
        for (int x = x0; x <= x1; ++x) {
            const double dx = (double)x - cx;
            if (dx * dx + dy * dy < r2) {
                if (cnt == 0) first = x;
                ++cnt;
            }
        }
    }
    // inclusive scan of the row counts over the surfel's lanes
    int incl = cnt;
#pragma unroll
    for (int o = 1; o < LANES; o <<= 1) {
        const int v = __shfl_up(incl, o, LANES);
        if (hl >= o) incl += v;
    }
    if (hl < d.nrows) {
        row_x0[hl] = first;
        row_start[hl + 1] = incl;
    }
    if (hl == 0) row_start[0] = 0;
    wave_sync();
    d.total = min(row_start[d.nrows], kWaveSize * kDiscPPL);
    return d;
}

// Pixel k (< total) of a disc.
__device__ __forceinline__ void disc_pixel(const DiscRows& d, const int* row_x0, const int* row_start,
                                           int k, int& x, int& y) {
    int i = 0;
    while (row_start[i + 1] <= k) ++i;
    x = row_x0[i] + (k - row_start[i]);
    y = d.y0 + i;
}

// Gauss-Newton over disc surfels: SPW surfels per wavefront, LANES = 64 /
// SPW lanes each (the batch's items are runs of SPW surfels of one keyframe),
// with the same per-pixel terms, frame loop, reduction and owner-lane step as
// the tile kernel, over the discs' pixels.  Each surfel's warp constants are
// anchored at the pixel nearest its centre.  With two surfels per wavefront
// the owner step (one lane per surfel) serves two surfels at once and the
// reductions span 32 lanes.  Six wavefronts per SIMD (80 VGPRs, and the LDS
// of six workgroups per CU): the few values that spill are read by the owner
// step once per iteration or by its double-precision fallback only.
template <typename T, int SPW, bool BY_ROW>
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(6, 8))) void disc_gn_kernel(
    const BatchHeader* __restrict__ hdr_, int total) {
    constexpr int LANES = kWaveSize / SPW;        // lanes per surfel
    constexpr int PPL = kDiscPPL * SPW;           // pixel slots per lane
    constexpr int WPB = kBlockThreads / kWaveSize;
    constexpr bool packed = DiscSlot<T>::packed;
    static_assert(kDiscMaxRows <= LANES, "a disc row per lane");
    const cptr<BatchHeader> hdr = (cptr<BatchHeader>)hdr_;
    const int lane = threadIdx.x & (kWaveSize - 1);
    const int wave = threadIdx.x >> 6;
    const int h = lane / LANES, hl = lane % LANES;       // surfel of the wave, lane within it
    int item_ = (int)blockIdx.x * WPB + wave;
    if (hdr->n_queues == kXcds) {
        // one share of the items per XCD (workgroups go to the XCDs in turn)
        const int share = (int)(blockIdx.x % (unsigned)kXcds);
        item_ = hdr->queues[share].begin + (int)(blockIdx.x / (unsigned)kXcds) * WPB + wave;
        if (item_ >= hdr->queues[share].end) item_ = total;
    }
    const int item = __builtin_amdgcn_readfirstlane(item_);
    if (item >= total) return;
    __shared__ float4 s_pairs[WPB][SPW][kMaxNbr * kPairWords / 4];
    __shared__ float4 s_state[WPB][SPW][ST_WORDS / 4];
    __shared__ float4 s_sums[WPB][SPW][SM_WORDS / 4];
    __shared__ int s_rows[WPB][SPW][kDiscRowWords];
    // each lane's pixels: offsets from the anchor and keyframe values
    __shared__ uint32_t s_pix[WPB][PPL][kWaveSize];
    __shared__ float s_val[WPB][packed ? 1 : PPL][kWaveSize];
    float* const pairs = (float*)s_pairs[wave][h];
    float* const lst = (float*)s_state[wave][h];
    float* const lsm = (float*)s_sums[wave][h];
    int* const row_x0 = s_rows[wave][h];
    int* const row_start = s_rows[wave][h] + kDiscMaxRows;

    const cptr<KfDev> kfs = (cptr<KfDev>)hdr->kfs;
    const int kidx = find_kf(kfs, hdr->n_kf, item, 0);
    const cptr<KfDev> Kd = kfs + kidx;
    const int sidx = (item - Kd->item_base) * SPW + h;
    const bool have = sidx < Kd->disc_count;         // an odd count leaves the last half empty
    const int iters = hdr->iters;
    const float hk = hdr->huber_k;
    const float kap2 = hdr->kappa_fp64 * hdr->kappa_fp64;
    const bool depth_only = hdr->depth_only != 0;
    const float lm0 = hdr->lm_lambda;
    const bool lm = lm0 > 0.f;
    const int W = Kd->width, H = Kd->height;
    const int nf = Kd->n_nbr;
    const float img_scale = Kd->img_scale;
    const unsigned pitch_b = (unsigned)Kd->nbr_pitch_b;
    const unsigned img_bytes = pitch_b * (unsigned)H;
    const unsigned wm1 = (unsigned)(W - 1), hm1 = (unsigned)(H - 1);
    const float fxk = Kd->fx, fyk = Kd->fy, cxk = Kd->cx, cyk = Kd->cy;
    const float ux = have ? ((gptr<float>)Kd->disc_ux)[sidx] : __builtin_nanf("");
    const float uy = have ? ((gptr<float>)Kd->disc_uy)[sidx] : __builtin_nanf("");

    wave_sync();
    const DiscRows d = disc_rows<LANES>(ux, uy, Kd->disc_r, W, H, hl, row_x0, row_start);
    // slot count: the larger of the wavefront's surfels, so the loop is uniform
    int nslots = (d.total + LANES - 1) / LANES;
    if constexpr (SPW == 2) nslots = max(nslots, __shfl_xor(nslots, 32));
    nslots = __builtin_amdgcn_readfirstlane(nslots);
    // anchor pixel (nearest the centre; any fixed point works for the local
    // warp coordinates)
    const int ax = (int)rint(fmin(fmax((double)ux, -1e6), 1e6));
    const int ay = (int)rint(fmin(fmax((double)uy, -1e6), 1e6));
    stage_pair_words(hdr->frames + Kd->frame_base, nf, hl, (double)ax, (double)ay, pairs);
    const uint64_t fr_bits = (uint64_t)(const void*)(hdr->frames + Kd->frame_base);
    const uint32_t fr_lo = __builtin_amdgcn_readfirstlane((uint32_t)fr_bits);
    const uint32_t fr_hi = __builtin_amdgcn_readfirstlane((uint32_t)(fr_bits >> 32));
    const cptr<FrameDev> fr = (cptr<FrameDev>)(((uint64_t)fr_hi << 32) | fr_lo);

    // this lane's pixels k = hl + LANES j, kept in LDS so that the slot loop
    // holds one pixel's terms in registers at a time
    const gptr<T> kimg = (gptr<T>)Kd->kf_img;
    const float kf_scale = Kd->kf_scale;
    for (int j = 0; j < nslots; ++j) {
        const int k = hl + LANES * j;
        uint32_t pk = 0u;
        float v = 0.f;
        if (k < d.total) {
            int x, y;
            disc_pixel(d, row_x0, row_start, k, x, y);
            const T raw = kimg[(unsigned)y * (unsigned)Kd->kf_pitch + (unsigned)x];
            pk = ((uint32_t)(x - ax) & 0xffu) | (((uint32_t)(y - ay) & 0xffu) << 8) | (slot_bits(raw) << 16);
            v = (float)raw * kf_scale;
        }
        s_pix[wave][j][lane] = pk;
        if constexpr (!packed) s_val[wave][j][lane] = v;
    }
    // r_u - r_s = (anchor offset + (anchor - u_s)) / f
    const float fox = (float)((double)ax - (double)ux), foy = (float)((double)ay - (double)uy);
    const float ifx = 1.f / fxk, ify = 1.f / fyk;

    // owner (lane 0 of each surfel): the surfel's state
    const bool owner = hl == 0;
    const float rsx = (ux - cxk) / fxk, rsy = (uy - cyk) / fyk;
    float id = 0.f, nx = 0.f, ny = 0.f, nz = -1.f;
    uint32_t flags = 0u;
    if (have) {
        id = ((gptr<float>)Kd->inv_depth)[sidx];
        nx = ((gptr<float>)Kd->nx)[sidx];
        ny = ((gptr<float>)Kd->ny)[sidx];
        nz = ((gptr<float>)Kd->nz)[sidx];
        flags = ((gptr<uint32_t>)Kd->flags)[sidx] & ~F_GN_BITS;
    }
    bool alive = have, updated = false;
    float cost_out = 0.f;
    int nv_out = 0;
    float lam = lm0;
    float b1x = 0.f, b1y = 0.f, b1z = 0.f, b2x = 0.f, b2y = 0.f, b2z = 0.f;

    for (int it = 0; it < iters; ++it) {
        const bool last = (it == iters - 1);
        if (owner) {
            const float c = nx * rsx + ny * rsy + nz;
            if (alive && fabsf(c) < 1e-6f) {
                flags |= F_DEGENERATE;
                alive = false;
                cost_out = 0.f;
                nv_out = 0;
            }
            tangent_basis(nx, ny, nz, b1x, b1y, b1z, b2x, b2y, b2z);
            lst[ST_ID] = id; lst[ST_NX] = nx; lst[ST_NY] = ny; lst[ST_NZ] = nz;
            lst[ST_B1X] = b1x; lst[ST_B1Y] = b1y; lst[ST_B1Z] = b1z;
            lst[ST_B2X] = b2x; lst[ST_B2Y] = b2y; lst[ST_B2Z] = b2z;
            lst[ST_INVC] = rcp_fast(c);
            lst[ST_RSX] = rsx; lst[ST_RSY] = rsy;
            lst[ST_ALIVE] = alive ? 1.f : 0.f;
        }
        wave_sync();
        {
            const float4 sa = *(const float4*)(lst + 0);
            const float4 sb = *(const float4*)(lst + 4);
            const float4 sc = *(const float4*)(lst + 8);
            const float2 sd = *(const float2*)(lst + 12);
            const float sid = sa.x, snx = sa.y, sny = sa.z;
            const float sb1x = sb.x, sb1y = sb.y, sb1z = sb.z;
            const float sb2x = sb.w, sb2y = sc.x, sb2z = sc.y, inv_c = sc.z, srsx = sc.w;
            const float srsy = sd.x;
            const bool salive = sd.y != 0.f;
            // the surfel's parts of sigma_u and g_u (see gn_kernel), formed
            // once per iteration; the depth-only ablation zeroes kk
            const float cnx = snx * inv_c, cny = sny * inv_c;
            const float kk = depth_only ? 0.f : sid * inv_c;
            const float k1x = kk * sb1x, k1y = kk * sb1y, k2x = kk * sb2x, k2y = kk * sb2y;
            const float q1 = kk * fmaf(sb1x, srsx, fmaf(sb1y, srsy, sb1z));
            const float q2 = kk * fmaf(sb2x, srsx, fmaf(sb2y, srsy, sb2z));
            float ph[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            float pnv = 0.f, pcs = 0.f;
            for (int j = 0; j < nslots; ++j) {
                const uint32_t pk = s_pix[wave][j][lane];
                const float bdx = (float)(int8_t)(pk & 0xffu), bdy = (float)(int8_t)((pk >> 8) & 0xffu);
                const float ikf = packed ? slot_value<T>(pk) * kf_scale : s_val[wave][packed ? 0 : j][lane];
                const bool pv = hl + LANES * j < d.total;
                const float drx = (bdx + fox) * ifx, dry = (bdy + foy) * ify;
                const float sigma = fmaf(cny, dry, cnx * drx);
                const float idu = fmaf(sid, sigma, sid);
                const float g0 = 1.f + sigma;
                const float g1 = fmaf(-sigma, q1, fmaf(k1y, dry, k1x * drx));
                const float g2 = fmaf(-sigma, q2, fmaf(k2y, dry, k2x * drx));
                const bool pix_ok = salive && pv && (idu > 0.f);
                float A = 0.f, B = 0.f, cst = 0.f;
                int nvl = 0;
                if (last || lm)
                    frame_loop<T, true, BY_ROW>(pairs, fr, nf, bdx, bdy, idu, pix_ok, pitch_b, img_bytes, wm1, hm1,
                                        ikf, hk, img_scale, A, B, cst, nvl);
                else
                    frame_loop<T, false, BY_ROW>(pairs, fr, nf, bdx, bdy, idu, pix_ok, pitch_b, img_bytes, wm1, hm1,
                                         ikf, hk, img_scale, A, B, cst, nvl);
                {
                    const float ag0 = A * g0, ag1 = A * g1, ag2 = A * g2;
                    ph[0] = fmaf(ag0, g0, ph[0]); ph[1] = fmaf(ag0, g1, ph[1]);
                    ph[2] = fmaf(ag0, g2, ph[2]); ph[3] = fmaf(ag1, g1, ph[3]);
                    ph[4] = fmaf(ag1, g2, ph[4]); ph[5] = fmaf(ag2, g2, ph[5]);
                    ph[6] = fmaf(B, g0, ph[6]); ph[7] = fmaf(B, g1, ph[7]); ph[8] = fmaf(B, g2, ph[8]);
                    pnv += (float)nvl;
                    pcs += cst;
                }
            }
            float s0, s1, s2, s3, s4;
            {
#pragma clang fp contract(off)
                const bool odd = (hl & 1) != 0;
                s0 = pair_sum<LANES>(ph[0], ph[1], odd);
                s1 = pair_sum<LANES>(ph[2], ph[3], odd);
                s2 = pair_sum<LANES>(ph[4], ph[5], odd);
                s3 = pair_sum<LANES>(ph[6], ph[7], odd);
                s4 = pair_sum<LANES>(ph[8], pnv, odd);
            }
            float cs = 0.f;
            if (last || lm) cs = group_sum<LANES>(pcs);
            if (hl < 2) {
                float* o = lsm + hl;
                o[0] = s0; o[2] = s1; o[4] = s2; o[6] = s3; o[8] = s4;
                if (hl == 0) o[SM_COST] = cs;
            }
        }
        wave_sync();
        bool cand = false;
        float id_c = 0.f, nx_c = 0.f, ny_c = 0.f, nz_c = 0.f, cost_here = 0.f;
        int nv = 0;
        if (owner)
            cand = owner_step(lsm, alive, last, depth_only, lm, kap2, lam, id, nx, ny, nz, b1x, b1y, b1z,
                              b2x, b2y, b2z, flags, cost_out, nv_out, nv, cost_here, id_c, nx_c, ny_c,
                              nz_c);
        if (lm) {
            float inv_cc = 0.f;
            bool cand_ok = cand;
            if (owner && cand) {
                const float cc = nx_c * rsx + ny_c * rsy + nz_c;
                if (fabsf(cc) < 1e-6f) {             // candidate plane contains r_s
                    flags |= F_REJECTED;
                    lam *= 10.f;
                    cand_ok = false;
                }
                inv_cc = rcp_fast(cc);
            }
            if (owner) {
                lst[ST_ID] = id_c; lst[ST_NX] = nx_c; lst[ST_NY] = ny_c; lst[ST_NZ] = nz_c;
                lst[ST_INVC] = inv_cc;
                lst[ST_ALIVE] = cand_ok ? 1.f : 0.f;
            }
            wave_sync();
            {
                const float4 sa = *(const float4*)(lst + 0);
                const float inv_c = lst[ST_INVC];
                const bool calive = lst[ST_ALIVE] != 0.f;
                float cst2 = 0.f;
                int nv2l = 0;
                for (int j = 0; j < nslots; ++j) {
                    const uint32_t pk = s_pix[wave][j][lane];
                    const float bdx = (float)(int8_t)(pk & 0xffu), bdy = (float)(int8_t)((pk >> 8) & 0xffu);
                    const float ikf = packed ? slot_value<T>(pk) * kf_scale : s_val[wave][packed ? 0 : j][lane];
                    const bool pv = hl + LANES * j < d.total;
                    const float drx = (bdx + fox) * ifx, dry = (bdy + foy) * ify;
                    const float sig = fmaf(sa.z * inv_c, dry, (sa.y * inv_c) * drx);
                    const float idu_c = fmaf(sa.x, sig, sa.x);
                    frame_cost<T, BY_ROW>(pairs, fr, nf, bdx, bdy, idu_c, calive && pv && (idu_c > 0.f), pitch_b,
                                  img_bytes, wm1, hm1, ikf, hk, img_scale, cst2, nv2l);
                }
                const float c2 = group_sum<LANES>(cst2);
                const int n2 = group_sum<LANES>(nv2l);
                if (hl == 0) {
                    lsm[SM_COST] = c2;
                    lsm[SM_NV] = __int_as_float(n2);
                }
            }
            wave_sync();
            if (owner && cand_ok) cand_ok = lm_accept(lsm[SM_COST], __float_as_int(lsm[SM_NV]), cost_here, nv, lam);
            cand = cand_ok;
        }
        if (owner && cand) {
            id = id_c;
            nx = nx_c; ny = ny_c; nz = nz_c;
            updated = true;
        }
    }
    if (owner && have) {
        ((gmut<float>)Kd->inv_depth)[sidx] = id;
        ((gmut<float>)Kd->nx)[sidx] = nx;
        ((gmut<float>)Kd->ny)[sidx] = ny;
        ((gmut<float>)Kd->nz)[sidx] = nz;
        ((gmut<uint32_t>)Kd->flags)[sidx] = flags;
        ((gmut<float>)Kd->cost)[sidx] = iters > 0 ? cost_out : 0.f;
        ((gmut<uint32_t>)Kd->nvalid)[sidx] = (uint32_t)(iters > 0 ? nv_out : 0);
        if (updated) ((gmut<uint32_t>)Kd->last_update)[sidx] = hdr->stamp;
    }
}

// Depth-buffered render (Inverse Depth Calculation section): every usable
// surfel (no DEGENERATE or UNINIT flag, finite centre, plane not through its
// centre ray) writes Eq. 3 into the pixels of its disc; the closest (largest
// id_u > 0) wins and equal values go to the lower index.  id_u is evaluated
// in double in the printed form of Eq. 3, id_u = (r_u . n) / ((r_s / id_s) . n).
//
// The render works in screen tiles of kRenderTile x kRenderTile pixels.  The
// usable surfels are binned to the tiles their disc's bounding box meets (a
// count, an exclusive scan of the counts over the tiles of the whole batch,
// a fill); then one workgroup per tile gives each pixel to a thread, which
// walks the tile's list keeping the largest value and the lowest index that
// reaches it.  The outcome does not depend on the list order, so the fill's
// atomics leave it deterministic, and the depth test needs no atomics.

// Table entry of global surfel g (largest surfel_base <= g among entries
// with surfels) or of global tile t (by tile_base).
__device__ __forceinline__ int render_item_of_surfel(const DiscRenderItem* tab, int n, int g) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid].surfel_base <= g) lo = mid; else hi = mid - 1;
    }
    return lo;        // entries without surfels share the next base and are never the largest
}
__device__ __forceinline__ int render_item_of_tile(const DiscRenderItem* tab, int n, int t) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid].tile_base <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void fill_int_kernel(int32_t* __restrict__ p, int n, int32_t v) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

// Pass 0 counts a usable surfel in each tile its disc's bounding box meets
// and stores its raster record; pass 1 (after the scan) writes it into those
// tiles' lists.  One thread per surfel.
template <int PASS>
__global__ __launch_bounds__(256) void disc_bin_kernel(const DiscRenderItem* __restrict__ tab, int n_items,
                                                       int total, DiscRaster* __restrict__ rec,
                                                       int32_t* __restrict__ count,
                                                       const int32_t* __restrict__ start,
                                                       int32_t* __restrict__ list) {
#pragma clang fp contract(off)
    const int g = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (g >= total) return;
    const DiscRenderItem& a = tab[render_item_of_surfel(tab, n_items, g)];
    const int s = g - a.surfel_base;
    if (a.flags[s] & (F_DEGENERATE | F_UNINIT)) return;
    const double cx = (double)a.ux[s], cy = (double)a.uy[s], r = (double)a.radius;
    if (!isfinite(cx) || !isfinite(cy)) return;
    const double n0 = a.nx[s], n1 = a.ny[s], n2 = a.nz[s], ids = a.inv_depth[s];
    const double rs0 = (cx - a.cx) / a.fx, rs1 = (cy - a.cy) / a.fy;
    if (fabs(n0 * rs0 + n1 * rs1 + n2 * 1.0) < 1e-6) return;
    const double xlo = fmax(0.0, ceil(cx - r)), xhi = fmin((double)(a.width - 1), floor(cx + r));
    const double ylo = fmax(0.0, ceil(cy - r)), yhi = fmin((double)(a.height - 1), floor(cy + r));
    if (!(xlo <= xhi) || !(ylo <= yhi)) return;
    if (PASS == 0) {
        const double ps0 = rs0 / ids, ps1 = rs1 / ids, ps2 = 1.0 / ids;
        rec[g] = DiscRaster{cx, cy, n0, n1, n2, ps0 * n0 + ps1 * n1 + ps2 * n2};
    }
    const int tx0 = (int)xlo / kRenderTile, tx1 = (int)xhi / kRenderTile;
    const int ty0 = (int)ylo / kRenderTile, ty1 = (int)yhi / kRenderTile;
    for (int ty = ty0; ty <= ty1; ++ty)
        for (int tx = tx0; tx <= tx1; ++tx) {
            const int t = a.tile_base + ty * a.tiles_x + tx;
            if (PASS == 0)
                atomicAdd(count + t, 1);
            else
                list[start[t] + atomicSub(count + t, 1) - 1] = g;
        }
}

// Exclusive scan of the tile counts into start[0 .. n] (start[n] = the total):
// blocks of 1024 scan their counts and report their sums, one block scans the
// sums (in chunks, with a carry) and writes the total, the sums are added
// back.
__device__ __forceinline__ int block_exclusive_scan(int v, int* s_w, int& block_total) {
    const int lane = threadIdx.x & (kWaveSize - 1), wave = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < kWaveSize; o <<= 1) {
        const int y = __shfl_up(x, o, kWaveSize);
        if (lane >= o) x += y;
    }
    if (lane == kWaveSize - 1) s_w[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int w = 0; w < (int)(blockDim.x / kWaveSize); ++w) {
            const int t = s_w[w];
            s_w[w] = acc;
            acc += t;
        }
        s_w[16] = acc;
    }
    __syncthreads();
    block_total = s_w[16];
    const int ex = s_w[wave] + x - v;
    __syncthreads();
    return ex;
}
__global__ __launch_bounds__(1024) void bin_scan_block_kernel(const int32_t* __restrict__ count,
                                                              int32_t* __restrict__ start,
                                                              int32_t* __restrict__ block_sum, int n) {
    __shared__ int s_w[17];
    const int i = (int)(blockIdx.x * 1024 + threadIdx.x);
    int tot;
    const int ex = block_exclusive_scan(i < n ? count[i] : 0, s_w, tot);
    if (i < n) start[i] = ex;
    if (threadIdx.x == 0) block_sum[blockIdx.x] = tot;
}
__global__ __launch_bounds__(1024) void bin_scan_top_kernel(int32_t* __restrict__ block_sum, int nb,
                                                            int32_t* __restrict__ start, int n) {
    __shared__ int s_w[17];
    int carry = 0;
    for (int c0 = 0; c0 < nb; c0 += 1024) {
        const int i = c0 + (int)threadIdx.x;
        int tot;
        const int ex = block_exclusive_scan(i < nb ? block_sum[i] : 0, s_w, tot);
        if (i < nb) block_sum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) start[n] = carry;
}
__global__ __launch_bounds__(1024) void bin_scan_add_kernel(int32_t* __restrict__ start,
                                                            const int32_t* __restrict__ block_sum, int n) {
    const int i = (int)(blockIdx.x * 1024 + threadIdx.x);
    if (i < n) start[i] += block_sum[blockIdx.x];
}

// One workgroup per tile, one thread per pixel: the largest Eq. 3 value over
// the tile's surfels whose disc holds the pixel, and the lowest index among
// those that reach it.  The tile's list is staged in LDS a workgroup-wide
// chunk at a time (one list entry and its raster record per thread, all
// loads in flight at once), so the per-pixel walk reads LDS instead of
// waiting on a dependent pair of loads per entry.
__global__ __launch_bounds__(kRenderTile * kRenderTile) void disc_raster_kernel(
    const DiscRenderItem* __restrict__ tab, int n_items, const DiscRaster* __restrict__ rec,
    const int32_t* __restrict__ start, const int32_t* __restrict__ list) {
#pragma clang fp contract(off)
    constexpr int kChunk = kRenderTile * kRenderTile;
    __shared__ DiscRaster s_rec[kChunk];
    __shared__ int s_idx[kChunk];
    const int t = (int)blockIdx.x;
    const DiscRenderItem& a = tab[render_item_of_tile(tab, n_items, t)];
    const int lt = t - a.tile_base;
    const int ty = lt / a.tiles_x, tx = lt - ty * a.tiles_x;
    const int x = tx * kRenderTile + (int)(threadIdx.x % kRenderTile);
    const int y = ty * kRenderTile + (int)(threadIdx.x / kRenderTile);
    const bool inside = x < a.width && y < a.height;
    const double xd = (double)x, yd = (double)y, r = (double)a.radius, r2 = r * r;
    const double ru0 = (xd - a.cx) / a.fx, ru1 = (yd - a.cy) / a.fy;
    unsigned long long best = 0ull;
    int who = 0x7fffffff;
    const int k0 = start[t], k1 = start[t + 1];
    for (int c0 = k0; c0 < k1; c0 += kChunk) {
        const int nc = min(kChunk, k1 - c0);
        __syncthreads();                     // the previous chunk is read
        if ((int)threadIdx.x < nc) {
            const int g = list[c0 + (int)threadIdx.x];
            s_idx[threadIdx.x] = g;
            s_rec[threadIdx.x] = rec[g];
        }
        __syncthreads();
        if (!inside) continue;
        for (int e = 0; e < nc; ++e) {
            const DiscRaster& q = s_rec[e];
            const double dx = xd - q.cx, dy = yd - q.cy;
            if (!(dx * dx + dy * dy < r2)) continue;
            const double v = (ru0 * q.n0 + ru1 * q.n1 + 1.0 * q.n2) / q.den;
            if (!(v > 0.0) || !isfinite(v)) continue;
            const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
            const int s = s_idx[e] - a.surfel_base;
            if (bits > best) {
                best = bits;
                who = s;
            } else if (bits == best && s < who) {
                who = s;
            }
        }
    }
    if (!inside) return;
    const size_t o = (size_t)y * (size_t)a.width + (size_t)x;
    a.inv_depth_out[o] = best ? (float)__longlong_as_double((long long)best) : 0.f;
    if (a.index_out) a.index_out[o] = best ? who : -1;
}

// Placement runs over a table of keyframes: candidates and new surfels are
// numbered keyframe after keyframe (cand_base, init_base); the entry owning
// number g is the last whose base is <= g (entries with none share the next
// base and are never the last).
__device__ __forceinline__ int place_entry_of_cand(const DiscPlaceArgs* tab, int n, int g) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid].cand_base <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}
__device__ __forceinline__ int place_entry_of_init(const DiscPlaceArgs* tab, int n, int g) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid].init_base <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// The search for empty areas (Surfel Initialization section): one wavefront
// per lattice candidate u_ns = (spacing/2 + i spacing, spacing/2 + j
// spacing), its lanes sharing the window of pixels within alpha r; the
// candidate qualifies when no non-empty pixel of the index map lies within
// alpha r (integer squared distance against (alpha r)^2 in double).
__global__ __launch_bounds__(kBlockThreads) void disc_search_kernel(const DiscPlaceArgs* __restrict__ tab,
                                                                    int n_items, int total) {
    const int lane = threadIdx.x & (kWaveSize - 1);
    const int g = __builtin_amdgcn_readfirstlane((int)blockIdx.x * (kBlockThreads / kWaveSize) +
                                                 (int)(threadIdx.x >> 6));
    if (g >= total) return;
    const DiscPlaceArgs& a = tab[place_entry_of_cand(tab, n_items, g)];
    const int c = g - a.cand_base;
    const int cx = a.spacing / 2 + (c % a.cand_x) * a.spacing;
    const int cy = a.spacing / 2 + (c / a.cand_x) * a.spacing;
    const double ar = (double)a.alpha * (double)a.radius;
    const double ar2 = ar * ar;
    const int reach = (int)floor(ar);
    const int side = 2 * reach + 1, npix = side * side;
    bool hit = false;
    for (int k0 = 0; k0 < npix; k0 += kWaveSize) {
        const int k = k0 + lane;
        if (k < npix) {
            const int dy = k / side - reach, dx = k % side - reach;
            const int x = cx + dx, y = cy + dy;
            if (x >= 0 && y >= 0 && x < a.width && y < a.height &&
                (double)(dx * dx + dy * dy) <= ar2 && a.index_map[(size_t)y * a.width + x] >= 0)
                hit = true;
        }
        if (__ballot(hit) != 0ull) break;     // wave-uniform
    }
    // the vote of the whole wavefront, taken before narrowing to one lane
    const bool empty = __ballot(hit) == 0ull;
    if (lane == 0) a.cand_flag[c] = empty ? 1 : 0;
}

// Placement: the qualifying candidates in lattice order become surfels
// first, first + 1, ... (as many as there is room for); counts[0] = placed,
// counts[1] = qualifying.  One workgroup per keyframe scans its flags in
// chunks.
__global__ __launch_bounds__(1024) void disc_compact_kernel(const DiscPlaceArgs* __restrict__ tab) {
    const DiscPlaceArgs& a = tab[blockIdx.x];
    __shared__ int s_wave[1024 / kWaveSize + 1];
    const int n = a.cand_x * a.cand_y;
    const int lane = threadIdx.x & (kWaveSize - 1);
    const int wave = threadIdx.x >> 6;
    constexpr int kWaves = 1024 / kWaveSize;
    int base = 0;
    for (int c0 = 0; c0 < n; c0 += 1024) {
        const int c = c0 + (int)threadIdx.x;
        const bool f = c < n && a.cand_flag[c] != 0;
        const unsigned long long ball = __ballot(f);
        const int below = __popcll(ball & ((1ull << lane) - 1ull));
        if (lane == 0) s_wave[wave] = __popcll(ball);
        __syncthreads();
        if (threadIdx.x == 0) {
            int acc = 0;
            for (int w = 0; w < kWaves; ++w) {
                const int t = s_wave[w];
                s_wave[w] = acc;
                acc += t;
            }
            s_wave[kWaves] = acc;
        }
        __syncthreads();
        const int rank = base + s_wave[wave] + below;
        if (f && rank < a.room) {
            const int cx = a.spacing / 2 + (c % a.cand_x) * a.spacing;
            const int cy = a.spacing / 2 + (c / a.cand_x) * a.spacing;
            a.ux[a.first + rank] = (float)cx;
            a.uy[a.first + rank] = (float)cy;
        }
        base += s_wave[kWaves];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.counts[0] = min(base, a.room);
        a.counts[1] = base;
    }
}

__device__ __forceinline__ int wave_min(int v) {
    for (int m = 1; m < kWaveSize; m <<= 1) v = min(v, __shfl_xor(v, m));
    return v;
}

// Neighbour initialisation of the placed surfels (Surfel Initialization
// section), one wavefront each: the neighbours are the surfels below
// `first` that own a pixel of the index map closer than beta r to the new
// centre, visited in index order (the wavefront finds the next smallest
// index each round); id = mean of Eq. 3 of their planes at the new ray,
// n = mean of their normals sign-aligned to the first, renormalised; none
// usable: UNINIT with id 0 and n = (0, 0, -1).
__global__ __launch_bounds__(kWaveSize) void disc_init_kernel(const DiscPlaceArgs* __restrict__ tab,
                                                              int n_items) {
    // the window's surfel indices (those within beta r, below `first`), or -1
    __shared__ int s_win[(2 * kDiscMaxWindowReach + 1) * (2 * kDiscMaxWindowReach + 1)];
    const int lane = threadIdx.x;
    const int g = __builtin_amdgcn_readfirstlane((int)blockIdx.x);
    const DiscPlaceArgs& a = tab[place_entry_of_init(tab, n_items, g)];
    const int w = g - a.init_base;
    if (w >= a.counts[0]) return;
    const int i = a.first + w;
    const int cx = (int)a.ux[i], cy = (int)a.uy[i];
    const double br = (double)a.beta * (double)a.radius;
    const double br2 = br * br;
    const int reach = (int)ceil(br);
    const int side = 2 * reach + 1, npix = side * side;
    for (int k = lane; k < npix; k += kWaveSize) {
        const int dy = k / side - reach, dx = k % side - reach;
        const int x = cx + dx, y = cy + dy;
        int j = -1;
        if (x >= 0 && y >= 0 && x < a.width && y < a.height && (double)(dx * dx + dy * dy) < br2) {
            j = a.index_map[(size_t)y * a.width + x];
            if (j >= a.first) j = -1;
        }
        s_win[k] = j;
    }
    wave_sync();
    const float rnx = ((float)cx - a.cx) / a.fx, rny = ((float)cy - a.cy) / a.fy;
    int last = -1, count = 0;
    float id_sum = 0.f, sx = 0.f, sy = 0.f, sz = 0.f, rx = 0.f, ry = 0.f, rz = 0.f;
    for (;;) {
        // next neighbour in index order
        int best = 0x7fffffff;
        for (int k = lane; k < npix; k += kWaveSize) {
            const int j = s_win[k];
            if (j > last) best = min(best, j);
        }
        const int j = __builtin_amdgcn_readfirstlane(wave_min(best));
        if (j == 0x7fffffff) break;
        last = j;
        if (a.flags[j] & (F_UNINIT | F_DEGENERATE)) continue;
        const float njx = a.nx[j], njy = a.ny[j], njz = a.nz[j];
        const float rjx = (a.ux[j] - a.cx) / a.fx, rjy = (a.uy[j] - a.cy) / a.fy;
        const float cj = njx * rjx + njy * rjy + njz;
        if (fabsf(cj) < 1e-6f) continue;
        // Eq. 3 of plane j at the new surfel's ray
        const float id = a.inv_depth[j] * (njx * rnx + njy * rny + njz) / cj;
        if (count == 0) { rx = njx; ry = njy; rz = njz; }
        const float sg = (njx * rx + njy * ry + njz * rz) < 0.f ? -1.f : 1.f;
        id_sum += id;
        sx += sg * njx; sy += sg * njy; sz += sg * njz;
        ++count;
    }
    if (lane != 0) return;
    bool ok = count > 0;
    float idn = 0.f, l2 = 0.f;
    if (ok) {
        const float inv = 1.0f / (float)count;
        idn = id_sum * inv;
        sx *= inv; sy *= inv; sz *= inv;
        l2 = sx * sx + sy * sy + sz * sz;
        ok = (l2 > 0.f) && (idn > 0.f) && isfinite(idn) && isfinite(l2);
    }
    if (ok) {
        const float il = 1.0f / sqrtf(l2);
        a.inv_depth[i] = idn;
        a.nx[i] = sx * il; a.ny[i] = sy * il; a.nz[i] = sz * il;
        a.flags[i] = 0u;
    } else {
        a.inv_depth[i] = 0.f;
        a.nx[i] = 0.f; a.ny[i] = 0.f; a.nz[i] = -1.f;
        a.flags[i] = F_UNINIT;
    }
    a.cost[i] = 0.f;
    a.nvalid[i] = 0u;
    a.last_update[i] = 0u;
}

// Eq. 10 for disc surfels (a disc stays a disc): a usable source surfel (no
// DEGENERATE or UNINIT flag, id_s > 0) moves to p' = R (r_s / id_s) + t with
// n' = R n and is re-centred at u' = K_dst pi(p'), inverse depth 1/p'_z.
// Those with p'_z > 0 and u' in [0, W-1] x [0, H-1] are written in source
// order (as many as there is room for).  One workgroup walks the sources in
// passes of kDiscXferSub chunks of 1024 (a thread's kDiscXferSub landings
// are independent, so their loads and double arithmetic overlap), ranks the
// pass's landings in source order with one scan over (chunk, wavefront)
// and writes them; every landing is computed in double in the oracle's
// order, so the kept set and the order are the same.
constexpr int kDiscXferSub = 4;
__global__ __launch_bounds__(1024) void disc_transfer_kernel(const DiscTransferArgs* __restrict__ tab) {
#pragma clang fp contract(off)
    const DiscTransferArgs& a = tab[blockIdx.x];          // one workgroup per keyframe pair
    constexpr int kWaves = 1024 / kWaveSize;
    constexpr int kSlots = kDiscXferSub * kWaves;         // (chunk, wavefront) in source order
    static_assert(kSlots <= kWaveSize, "one wavefront scans the slots");
    __shared__ int s_cnt[kSlots + 1];
    const int lane = threadIdx.x & (kWaveSize - 1);
    const int wave = threadIdx.x >> 6;
    int base = 0;
    for (int c0 = 0; c0 < a.count; c0 += 1024 * kDiscXferSub) {
        bool land[kDiscXferSub];
        float fu[kDiscXferSub], fv[kDiscXferSub], fid[kDiscXferSub];
        float f0[kDiscXferSub], f1[kDiscXferSub], f2[kDiscXferSub];
        int below[kDiscXferSub];
#pragma unroll
        for (int j = 0; j < kDiscXferSub; ++j) {
            const int k = c0 + j * 1024 + (int)threadIdx.x;
            land[j] = false;
            double u = 0.0, v = 0.0, idn = 0.0, m0 = 0.0, m1 = 0.0, m2 = 0.0;
            if (k < a.count && !(a.flags[k] & (F_DEGENERATE | F_UNINIT)) && a.inv_depth[k] > 0.f) {
                const double ids = a.inv_depth[k];
                const double rs0 = ((double)a.ux[k] - a.sK[2]) / a.sK[0];
                const double rs1 = ((double)a.uy[k] - a.sK[3]) / a.sK[1];
                const double p0 = rs0 / ids, p1 = rs1 / ids, p2 = 1.0 / ids;
                const double n0 = a.nx[k], n1 = a.ny[k], n2 = a.nz[k];
                const double q0 = a.R[0] * p0 + a.R[1] * p1 + a.R[2] * p2 + a.t[0];
                const double q1 = a.R[3] * p0 + a.R[4] * p1 + a.R[5] * p2 + a.t[1];
                const double q2 = a.R[6] * p0 + a.R[7] * p1 + a.R[8] * p2 + a.t[2];
                m0 = a.R[0] * n0 + a.R[1] * n1 + a.R[2] * n2;
                m1 = a.R[3] * n0 + a.R[4] * n1 + a.R[5] * n2;
                m2 = a.R[6] * n0 + a.R[7] * n1 + a.R[8] * n2;
                if (q2 > 0.0) {
                    u = a.dK[0] * (q0 / q2) + a.dK[2];
                    v = a.dK[1] * (q1 / q2) + a.dK[3];
                    land[j] = u >= 0.0 && u <= (double)(a.dst_w - 1) && v >= 0.0 && v <= (double)(a.dst_h - 1);
                    idn = 1.0 / q2;
                }
            }
            // the stored values (rounded to float here rather than at the store)
            fu[j] = (float)u; fv[j] = (float)v; fid[j] = (float)idn;
            f0[j] = (float)m0; f1[j] = (float)m1; f2[j] = (float)m2;
            const unsigned long long ball = __ballot(land[j]);
            below[j] = __popcll(ball & ((1ull << lane) - 1ull));
            if (lane == 0) s_cnt[j * kWaves + wave] = __popcll(ball);
        }
        __syncthreads();
        if (wave == 0) {
            // exclusive scan of the slot counts (slot = lane), total in s_cnt[kSlots]
            const int c = lane < kSlots ? s_cnt[lane] : 0;
            int incl = c;
#pragma unroll
            for (int d = 1; d < kWaveSize; d <<= 1) {
                const int t = __shfl_up(incl, d);
                if (lane >= d) incl += t;
            }
            if (lane < kSlots) s_cnt[lane] = incl - c;
            if (lane == kWaveSize - 1) s_cnt[kSlots] = incl;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kDiscXferSub; ++j) {
            const int k = c0 + j * 1024 + (int)threadIdx.x;
            const int rank = base + s_cnt[j * kWaves + wave] + below[j];
            if (land[j] && rank < a.capacity) {
                a.dst.inv_depth[rank] = fid[j];
                a.dst.nx[rank] = f0[j];
                a.dst.ny[rank] = f1[j];
                a.dst.nz[rank] = f2[j];
                a.dst.flags[rank] = 0u;
                a.dst.cost[rank] = 0.f;
                a.dst.nvalid[rank] = 0u;
                a.dst.last_update[rank] = a.last_update[k];
                a.dux[rank] = fu[j];
                a.duy[rank] = fv[j];
                if (a.src_index) a.src_index[rank] = k;
            }
        }
        base += s_cnt[kSlots];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.counts[0] = min(base, a.capacity);
        a.counts[1] = base;
    }
}

hipError_t launch_disc_transfer(const DiscTransferArgs* table, int n_pairs, hipStream_t s) {
    disc_transfer_kernel<<<n_pairs, 1024, 0, s>>>(table);
    return hipGetLastError();
}

template <bool R>
static void launch_disc_gn_rows(int dtype, const BatchHeader* hdr, int total_items, dim3 grid, hipStream_t s) {
    if (dtype == 0)
        disc_gn_kernel<float, disc_surfels_per_wave(0), R><<<grid, kBlockThreads, 0, s>>>(hdr, total_items);
    else if (dtype == 1)
        disc_gn_kernel<_Float16, disc_surfels_per_wave(1), R><<<grid, kBlockThreads, 0, s>>>(hdr, total_items);
    else
        disc_gn_kernel<uint8_t, disc_surfels_per_wave(2), R><<<grid, kBlockThreads, 0, s>>>(hdr, total_items);
}

hipError_t launch_disc_gn(int dtype, const BatchHeader* hdr, int total_items, int grid_blocks, bool by_row,
                          hipStream_t s) {
    if (total_items <= 0) return hipSuccess;
    const dim3 grid(grid_blocks);
    if (by_row) launch_disc_gn_rows<true>(dtype, hdr, total_items, grid, s);
    else launch_disc_gn_rows<false>(dtype, hdr, total_items, grid, s);
    return hipGetLastError();
}

hipError_t launch_disc_render(const DiscRenderItem* table, int n_items, int total_surfels, int total_tiles,
                              const DiscRenderScratch& w, hipStream_t s) {
    const int nb = (total_tiles + 1023) / 1024;
    fill_int_kernel<<<std::min((total_tiles + 255) / 256, 4096), 256, 0, s>>>(w.count, total_tiles, 0);
    const int sblocks = (total_surfels + 255) / 256;
    if (total_surfels > 0)
        disc_bin_kernel<0><<<sblocks, 256, 0, s>>>(table, n_items, total_surfels, w.rec, w.count, w.start,
                                                   w.list);
    bin_scan_block_kernel<<<nb, 1024, 0, s>>>(w.count, w.start, w.block_sum, total_tiles);
    bin_scan_top_kernel<<<1, 1024, 0, s>>>(w.block_sum, nb, w.start, total_tiles);
    bin_scan_add_kernel<<<nb, 1024, 0, s>>>(w.start, w.block_sum, total_tiles);
    if (total_surfels > 0)
        disc_bin_kernel<1><<<sblocks, 256, 0, s>>>(table, n_items, total_surfels, w.rec, w.count, w.start,
                                                   w.list);
    disc_raster_kernel<<<total_tiles, kRenderTile * kRenderTile, 0, s>>>(table, n_items, w.rec, w.start,
                                                                         w.list);
    return hipGetLastError();
}

hipError_t launch_disc_place(const DiscPlaceArgs* table, int n_items, int total_cands, int total_init,
                             hipStream_t s) {
    const int waves = kBlockThreads / kWaveSize;
    if (total_cands > 0)
        disc_search_kernel<<<(total_cands + waves - 1) / waves, kBlockThreads, 0, s>>>(table, n_items,
                                                                                        total_cands);
    disc_compact_kernel<<<n_items, 1024, 0, s>>>(table);
    if (total_init > 0) disc_init_kernel<<<total_init, kWaveSize, 0, s>>>(table, n_items);
    return hipGetLastError();
}

}  // namespace sgn
