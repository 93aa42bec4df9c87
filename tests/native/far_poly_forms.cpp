// Host check of the stage kernels' inline far side across a hanging face
// to finer neighbours (far_poly, LINK_FINE: the combine of Eq. 17 with the
// 2^d children unrolled and the table's zero entries skipped) against the
// same combine written as a loop over the children that multiplies every
// table entry (the form that once replaced it and was withdrawn after a
// degree-3 GPU run returned NaN).  Both are compiled for the host from the
// kernels' own header and evaluated on random states for every face axis,
// side and face point at degrees 1..3 in 2-D and 3-D, N = 4.  For finite
// inputs the two must agree bit for bit: the same products summed in the
// same order (a skipped zero term leaves the sum unchanged).  Prints the
// number of compared values and "OK"; exits non-zero on a difference.
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "../../paper_2502_12620_amd/csrc/kernels.hpp"

using namespace dgk;

template <int D, int P, int A, int NV>
static void loop_form(const StageArgs &g, int side, int t, const FaceLink &L, double (&Kf)[NV][Tab<D, P>::NB])
{
    constexpr int NB = Tab<D, P>::NB;
    const int N = g.N, ncell = D == 2 ? N * N : N * N * N;
    const long sv = long(NB) * ncell;
    const double *fk = g.us + long(link_nbr(L, fine_block(t, N, D))) * NV * sv;
    for (int v = 0; v < NV; ++v)
        for (int m = 0; m < NB; ++m) Kf[v][m] = 0.0;
    for (int ch = 0; ch < (1 << D); ++ch) {
        const int fc = fine_cell(A, side, t, ch, N, D);
        for (int v = 0; v < NV; ++v) {
            double kv[NB];
            for (int n = 0; n < NB; ++n) kv[n] = fk[v * sv + n * ncell + fc];
            for (int m = 0; m < NB; ++m)
                for (int n = 0; n < NB; ++n) Kf[v][m] = fma(kTab<D, P>.comb[ch][m][n], kv[n], Kf[v][m]);
        }
    }
}

static long compared = 0;

template <int D, int P, int A>
static int check_axis(const StageArgs &g, const FaceLink &L)
{
    constexpr int NV = D + 2, NB = Tab<D, P>::NB;
    const int N = g.N, nfc = D == 2 ? N : N * N;
    double K[NV][NB] = {};
    for (int side = -1; side <= 1; side += 2)
        for (int t = 0; t < nfc; ++t) {
            double a[NV][NB], b[NV][NB];
            far_poly<D, P, A, GUARD_INLINE, NV, double>(g, K, 0, side, t, L, a);
            loop_form<D, P, A, NV>(g, side, t, L, b);
            if (std::memcmp(a, b, sizeof(a)) != 0) {
                std::fprintf(stderr, "DIFFERENT: dim %d degree %d axis %d side %d t %d\n", D, P, A, side, t);
                return 1;
            }
            compared += NV * NB;
        }
    return 0;
}

template <int D, int P>
static int check()
{
    constexpr int NV = D + 2, NB = Tab<D, P>::NB;
    const int N = 4, ncell = D == 2 ? N * N : N * N * N, nleaves = 1 + (1 << (D - 1));
    std::vector<double> us(size_t(nleaves) * NV * NB * ncell);
    std::mt19937_64 rng(2502 + 10 * D + P);
    std::normal_distribution<double> nd(0.0, 1.0);
    for (auto &x : us) x = nd(rng);
    StageArgs g{};
    g.us = us.data();
    g.N = N;
    g.nleaves = nleaves;
    FaceLink L{};
    L.type = dgamr::LINK_FINE;
    for (int k = 0; k < 4; ++k) L.nbr[k] = k < (1 << (D - 1)) ? 1 + k : 0;
    int bad = check_axis<D, P, 0>(g, L) | check_axis<D, P, 1>(g, L);
    if constexpr (D == 3) bad |= check_axis<D, P, 2>(g, L);
    return bad;
}

int main()
{
    int bad = check<2, 1>() | check<2, 2>() | check<2, 3>() | check<3, 1>() | check<3, 2>() | check<3, 3>();
    if (bad) return 1;
    std::printf("OK %ld far-side coefficients compared\n", compared);
    return 0;
}
