// Volume integral of the FP32 residual on the matrix cores (gfx950
// v_mfma_f32_16x16x4f32, FP32 inputs and accumulation).
//
// The thread-per-cell stage kernel holds one cell's coefficients K[v][m]
// per lane.  A wave's 64 cells are handled as four tiles of 16 cells; for
// each tile and each block of 16 quadrature points the two contractions of
// the volume integral (Sec. 2, Eq. 3-4) become matrix products with the
// cells as the 16 columns:
//   evaluate  U^T[q][c]  = sum_m  B[q][m]   K^T[m][c]      (B = phi_m(xi_q))
//   project   R^T[m][c] += sum_q  Dp_a[m][q] F_a^T[q][c]   (Dp_a = w_q dphi_m/dxi_a / M_m)
// with the Euler flux F_a evaluated pointwise between them, on the vector
// unit, in the lanes that hold each point's state.  Operand layout of the
// 16x16x4 instruction: lane l supplies A[l%16][l/16] and B[l/16][l%16], and
// holds D[4 (l/16) + r][l%16] in its register r.  The evaluate's result
// therefore gives lane l the points q = 16 pb + 4 (l/16) + r of cell l%16,
// which is exactly the B operand of the project when its K steps take the
// points in that order (K step r, K index l/16), so no transpose is needed
// between the two.  K^T comes from LDS (each lane writes its own cell's
// coefficients; a wave only reads its own cells, so no barrier), and the
// tile's R^T goes back through the same LDS slots to the lanes that own
// the cells.
#pragma once

#include "kernels.hpp"

namespace dgk {

typedef float mf_floatx4 __attribute__((ext_vector_type(4)));

// whether the FP32 thread-per-cell stage kernel contracts its volume
// integral on the matrix cores: degree >= 2, where the basis matrices are
// dense enough (16x16 tiles of 6 to 10 modes and 9 to 27 points).  Not at
// 3-D degree 3: there the fused kernel with the matrix-core volume needs
// 512 VGPR + AGPR and about 1.2 KB of scratch per lane, and its fused step
// with conservative mortars returned non-finite values in a parity test
// whose residual-only form (no spills) matched; the 3-D degree-3 FP32
// residual stays on the vector unit.
template <int D, int P>
constexpr bool mfma_volume() { return P >= 2 && !(D == 3 && P == 3); }

// Per-lane A operands of both contractions, zero-padded to whole tiles.
template <int D, int P>
struct MfmaTab {
    static constexpr int NB = Tab<D, P>::NB, NQ = Tab<D, P>::NQ;
    static constexpr int NBP = (NB + 3) / 4 * 4; // modes padded to K steps of 4
    static constexpr int NKS = NBP / 4;
    static constexpr int NPB = (NQ + 15) / 16;   // blocks of 16 points
    static constexpr int NMB = (NB + 15) / 16;   // blocks of 16 modes
    float ev[NPB][NKS][64] = {};          // B[q = 16 pb + l%16][m = 4 ks + l/16]
    float pr[D][NPB][4][NMB][64] = {};    // Dp_a[m = 16 mb + l%16][q = 16 pb + 4 (l/16) + r]
    constexpr MfmaTab()
    {
        for (int pb = 0; pb < NPB; ++pb)
            for (int l = 0; l < 64; ++l) {
                for (int ks = 0; ks < NKS; ++ks) {
                    const int q = 16 * pb + l % 16, m = 4 * ks + l / 16;
                    ev[pb][ks][l] = (q < NQ && m < NB) ? float(kTab<D, P>.phi_v[q][m]) : 0.0f;
                }
                for (int a = 0; a < D; ++a)
                    for (int r = 0; r < 4; ++r)
                        for (int mb = 0; mb < NMB; ++mb) {
                            const int q = 16 * pb + 4 * (l / 16) + r, m = 16 * mb + l % 16;
                            pr[a][pb][r][mb][l] = (q < NQ && m < NB) ? float(kTab<D, P>.dproj[a][q][m]) : 0.0f;
                        }
            }
    }
};
template <int D, int P>
inline constexpr MfmaTab<D, P> kMfTab{};

// floats of LDS one wave needs
template <int D, int P>
constexpr int mfma_lds_floats() { return (D + 2) * MfmaTab<D, P>::NBP * 64; }

// R[v][m] += volume integral of the lane's cell.  lds: this wave's region
// of mfma_lds_floats() floats, free on entry and on return.  All 64 lanes
// of the wave take part.
template <int D, int P>
__device__ __forceinline__ void volume_mfma(const float (&K)[D + 2][Tab<D, P>::NB], float (&R)[D + 2][Tab<D, P>::NB],
                                            float *lds, const float *scale, float gm1)
{
    using MT = MfmaTab<D, P>;
    constexpr int NV = D + 2, NB = MT::NB, NQ = MT::NQ, NBP = MT::NBP, NKS = MT::NKS, NPB = MT::NPB, NMB = MT::NMB;
    const int lane = int(threadIdx.x) & 63, lo = lane & 15, hi = lane >> 4;
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int m = 0; m < NBP; ++m) lds[(v * NBP + m) * 64 + lane] = m < NB ? K[v][m] : 0.0f;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll 1
    for (int t = 0; t < 4; ++t) {
        const int cell = 16 * t + lo; // the tile's cell this lane computes for
        mf_floatx4 acc[NV][NMB];
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int mb = 0; mb < NMB; ++mb) acc[v][mb] = mf_floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 1
        for (int pb = 0; pb < NPB; ++pb) {
            // evaluate: U at the points 16 pb + 4 hi + r of `cell`
            mf_floatx4 u[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) u[v] = mf_floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int ks = 0; ks < NKS; ++ks) {
                const float a = kMfTab<D, P>.ev[pb][ks][lane];
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const float b = lds[(v * NBP + 4 * ks + hi) * 64 + cell];
                    u[v] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, u[v], 0, 0, 0);
                }
            }
            // pointwise Euler fluxes (Eq. 2, 23), scaled by 2/h_a; zero at the
            // padding points
            float F[D][NV][4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const bool live = 16 * pb + 4 * hi + r < NQ;
                float U[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) U[v] = live ? u[v][r] : (v == 0 ? 1.0f : 0.0f);
                const float rinv = recip(U[0]);
                const float p = pressure_r<D, float>(U, gm1, rinv);
                static_for<0, D>([&](auto Ai) __attribute__((always_inline)) {
                    constexpr int A = Ai;
                    float Fa[NV];
                    euler_flux<D, A, float>(U, U[1 + A] * rinv, p, Fa);
#pragma unroll
                    for (int v = 0; v < NV; ++v) F[A][v][r] = live ? Fa[v] * scale[A] : 0.0f;
                });
            }
            // project: K step r takes the points 16 pb + 4 k + r, k = l/16
#pragma unroll
            for (int a = 0; a < D; ++a)
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int mb = 0; mb < NMB; ++mb) {
                        const float A = kMfTab<D, P>.pr[a][pb][r][mb][lane];
#pragma unroll
                        for (int v = 0; v < NV; ++v)
                            acc[v][mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(A, F[a][v][r], acc[v][mb], 0, 0, 0);
                    }
        }
        // the tile's R^T into the LDS slots of its cells (their K has been
        // read): lane l holds modes 16 mb + 4 hi + r of `cell`
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int m = 16 * mb + 4 * hi + r;
                    if (m < NB) lds[(v * NBP + m) * 64 + cell] = acc[v][mb][r];
                }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int m = 0; m < NB; ++m) R[v][m] += lds[(v * NBP + m) * 64 + lane];
}

} // namespace dgk
