// Compile-time basis and quadrature tables for the DG kernels.
//
// Basis (Sec. 2, "P^K"): total-degree products of unnormalised Legendre
// polynomials on [-1,1]^d, |m| <= p, in graded order (|m| ascending, then
// m_x descending, then m_y descending).  Volume and face integrals use
// Gauss-Legendre rules with Q = p+1 points per axis; initial-condition
// projection uses p+3.  Everything here is a constant expression, so the
// fully unrolled kernels see every table entry as an immediate and skip
// structural zeros (e.g. d/dx of a mode without an x factor).
#pragma once

#include <cstdint>
#include <utility>

#ifndef DG_HD
#define DG_HD __host__ __device__
#endif

namespace dgk {

// ---- compile-time loops: the body receives std::integral_constant<int, I>
template <int B, int E, class F>
DG_HD __attribute__((always_inline)) inline void static_for(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(static_cast<F &&>(f));
    }
}

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

constexpr int num_modes(int d, int p)
{
    int n = 0;
    for (int s = 0; s <= p; ++s) n += (d == 2) ? (s + 1) : (s + 1) * (s + 2) / 2;
    return n;
}

// Gauss-Legendre nodes (ascending) and weights, closed forms / standard
// values for 1..6 points.
constexpr double gl_x(int q, int i)
{
    constexpr double x2[] = {-0.57735026918962576451, 0.57735026918962576451};
    constexpr double x3[] = {-0.77459666924148337704, 0.0, 0.77459666924148337704};
    constexpr double x4[] = {-0.86113631159405257522, -0.33998104358485626480, 0.33998104358485626480,
                             0.86113631159405257522};
    constexpr double x5[] = {-0.90617984593866399280, -0.53846931010568309104, 0.0, 0.53846931010568309104,
                             0.90617984593866399280};
    constexpr double x6[] = {-0.93246951420315202781, -0.66120938646626451366, -0.23861918608319690863,
                             0.23861918608319690863, 0.66120938646626451366, 0.93246951420315202781};
    return q == 1 ? 0.0 : q == 2 ? x2[i] : q == 3 ? x3[i] : q == 4 ? x4[i] : q == 5 ? x5[i] : x6[i];
}

constexpr double gl_w(int q, int i)
{
    constexpr double w2[] = {1.0, 1.0};
    constexpr double w3[] = {0.55555555555555555556, 0.88888888888888888889, 0.55555555555555555556};
    constexpr double w4[] = {0.34785484513745385737, 0.65214515486254614263, 0.65214515486254614263,
                             0.34785484513745385737};
    constexpr double w5[] = {0.23692688505618908751, 0.47862867049936646804, 0.56888888888888888889,
                             0.47862867049936646804, 0.23692688505618908751};
    constexpr double w6[] = {0.17132449237917034504, 0.36076157304813860757, 0.46791393457269104739,
                             0.46791393457269104739, 0.36076157304813860757, 0.17132449237917034504};
    return q == 1 ? 2.0 : q == 2 ? w2[i] : q == 3 ? w3[i] : q == 4 ? w4[i] : q == 5 ? w5[i] : w6[i];
}

// Legendre P_n and P_n' by the three-term recurrences
constexpr double leg(int n, double x)
{
    double a = 1.0, b = x;
    if (n == 0) return 1.0;
    for (int k = 1; k < n; ++k) {
        double c = ((2 * k + 1) * x * b - k * a) / (k + 1);
        a = b;
        b = c;
    }
    return b;
}

constexpr double dleg(int n, double x)
{
    // P'_{k+1} = P'_{k-1} + (2k+1) P_k
    if (n == 0) return 0.0;
    double a = 0.0, b = 1.0;
    for (int k = 1; k < n; ++k) {
        double c = a + (2 * k + 1) * leg(k, x);
        a = b;
        b = c;
    }
    return b;
}

// 1-D Legendre prolongation onto half intervals: child `hi` (0 lower half,
// 1 upper half), S1[a][c] = (2a+1)/2 int_{-1}^{1} P_a(t) P_c((t + s)/2) dt,
// s = -1 / +1; exact with 4 Gauss points for degrees <= 3.
constexpr double split1(int hi, int a, int c)
{
    double s = hi ? 1.0 : -1.0, acc = 0.0;
    for (int i = 0; i < 4; ++i) acc += gl_w(4, i) * leg(a, gl_x(4, i)) * leg(c, 0.5 * (gl_x(4, i) + s));
    return 0.5 * (2 * a + 1) * acc;
}

template <int D, int P>
struct Tab {
    static constexpr int NB = num_modes(D, P);
    static constexpr int NV = D + 2;
    static constexpr int Q = P + 1;
    static constexpr int NQ = ipow(Q, D);
    static constexpr int NF = ipow(Q, D - 1);

    int e[NB][3] = {};
    double inv_mass[NB] = {};       // prod (2 m_a + 1)/2
    double phi_v[NQ][NB] = {};      // phi_m at volume point q
    double dproj[D][NQ][NB] = {};   // w_q dphi_m/dxi_a (xi_q) / M_m
    double phi_f[D][NF][NB] = {};   // phi_m at the face point, xi_a = +1 (the -1 face adds (-1)^{m_a})
    double lift_f[D][NF][NB] = {};  // w_fq phi_m(face point, xi_a = +1) / M_m
    double split[1 << D][NB][NB] = {}; // child c: coefficients of the child from the parent (Eq. 11-12)
    double comb[1 << D][NB][NB] = {};  // child c's contribution to the parent (Eq. 13-14)

    constexpr Tab()
    {
        int n = 0;
        for (int s = 0; s <= P; ++s)
            for (int mx = s; mx >= 0; --mx) {
                if (D == 2) {
                    e[n][0] = mx;
                    e[n][1] = s - mx;
                    e[n][2] = 0;
                    ++n;
                } else {
                    for (int my = s - mx; my >= 0; --my) {
                        e[n][0] = mx;
                        e[n][1] = my;
                        e[n][2] = s - mx - my;
                        ++n;
                    }
                }
            }
        for (int m = 0; m < NB; ++m) {
            double im = 1.0;
            for (int a = 0; a < D; ++a) im *= 0.5 * (2 * e[m][a] + 1);
            inv_mass[m] = im;
        }
        for (int q = 0; q < NQ; ++q) {
            int qi[3] = {q % Q, (q / Q) % Q, q / (Q * Q)};
            double w = 1.0;
            for (int a = 0; a < D; ++a) w *= gl_w(Q, qi[a]);
            for (int m = 0; m < NB; ++m) {
                double v = 1.0;
                for (int a = 0; a < D; ++a) v *= leg(e[m][a], gl_x(Q, qi[a]));
                phi_v[q][m] = v;
                for (int ax = 0; ax < D; ++ax) {
                    double dv = 1.0;
                    for (int a = 0; a < D; ++a)
                        dv *= (a == ax) ? dleg(e[m][a], gl_x(Q, qi[a])) : leg(e[m][a], gl_x(Q, qi[a]));
                    dproj[ax][q][m] = w * dv * inv_mass[m];
                }
            }
        }
        for (int ax = 0; ax < D; ++ax)
            for (int f = 0; f < NF; ++f) {
                // tangential axes in increasing order, lower one fastest
                int t0 = f % Q, t1 = f / Q;
                double w = gl_w(Q, t0) * (D == 3 ? gl_w(Q, t1) : 1.0);
                for (int m = 0; m < NB; ++m) {
                    double v = 1.0;
                    int k = 0;
                    for (int a = 0; a < D; ++a) {
                        if (a == ax) continue;
                        v *= leg(e[m][a], gl_x(Q, k == 0 ? t0 : t1));
                        ++k;
                    }
                    phi_f[ax][f][m] = v;
                    lift_f[ax][f][m] = w * v * inv_mass[m];
                }
            }
        for (int c = 0; c < (1 << D); ++c)
            for (int m = 0; m < NB; ++m)
                for (int n2 = 0; n2 < NB; ++n2) {
                    double v = 1.0;
                    for (int a = 0; a < D; ++a) v *= split1((c >> a) & 1, e[m][a], e[n2][a]);
                    split[c][m][n2] = v;
                }
        // combine: C_c = 2^-d D^-1 S_c^T D with D = diag(reference mass)
        for (int c = 0; c < (1 << D); ++c)
            for (int m = 0; m < NB; ++m)
                for (int n2 = 0; n2 < NB; ++n2)
                    comb[c][m][n2] = split[c][n2][m] * inv_mass[m] / inv_mass[n2] / double(1 << D);
    }
};

template <int D, int P>
inline constexpr Tab<D, P> kTab{};

} // namespace dgk
