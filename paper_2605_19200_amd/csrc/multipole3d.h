// Host side of the 3D far field at any order (Eq. taylor carried past the
// paper's order 2).
//
// With 1/|x - q| = sum_{l,m} I_l^m(q - c) conj(R_l^m(x - c)) for |x - c| <
// |q - c| (regular / irregular solid harmonics below), the solid angle of a
// cluster, -integral n . grad_x (1/|x - q|) dA, equals
//   sum_{l >= 1} [ I_l^0 N_l^0 + 2 sum_{m >= 1} Re(I_l^m N_l^m) ],
//   N_l^m = - integral n . conj(grad R_l^m(x - c)) dA.
// R_l^m is a homogeneous polynomial of degree l, so truncating at l <= p + 1
// keeps exactly the terms of the order-p Taylor expansion of the integrand
// about c: the same expansion as Eq. taylor, evaluated through harmonics.
//
// Conventions (no Condon-Shortley phase), d = (x, y, z), rho^2 = |d|^2:
//   R_0^0 = 1,  R_m^m = R_{m-1}^{m-1} (x + i y) / (2m),
//   R_l^m = ((2l - 1) z R_{l-1}^m - rho^2 R_{l-2}^m) / ((l - m)(l + m)),
//   R_l^{-m} = (-1)^m conj(R_l^m);
// with these, R_l^m(a + b) = sum_{j, k} R_j^k(a) R_{l-j}^{m-k}(b), which
// translates the moments from a child's centre to its parent's (M2M).
#pragma once

#include <complex>
#include <cstring>

#include "gwn_internal.h"

namespace gwn {

inline int mp_index(int l, int m) { return l * (l + 1) / 2 - 1 + m; }

using cplx = std::complex<double>;

// R_l^m(d) and grad R_l^m(d) for 0 <= m <= l <= L (forward differentiation of
// the recurrences).
inline void regular_harmonics(const double d[3], int L, cplx R[kMaxLTail3 + 1][kMaxLTail3 + 1],
                              cplx dR[kMaxLTail3 + 1][kMaxLTail3 + 1][3])
{
    const double x = d[0], y = d[1], z = d[2];
    const double rho2 = x * x + y * y + z * z;
    const cplx xi(x, y);
    const cplx dxi[3] = {cplx(1, 0), cplx(0, 1), cplx(0, 0)};
    for (int m = 0; m <= L; ++m) {
        if (m == 0) {
            R[0][0] = 1.0;
            for (int a = 0; a < 3; ++a) dR[0][0][a] = 0.0;
        } else {
            const double f = 1.0 / (2 * m);
            R[m][m] = R[m - 1][m - 1] * xi * f;
            for (int a = 0; a < 3; ++a) dR[m][m][a] = (dR[m - 1][m - 1][a] * xi + R[m - 1][m - 1] * dxi[a]) * f;
        }
        for (int l = m + 1; l <= L; ++l) {
            const double den = 1.0 / ((double)(l - m) * (l + m));
            const cplx a1 = R[l - 1][m];
            const cplx a2 = l - 2 >= m ? R[l - 2][m] : cplx(0, 0);
            const double c1 = (2.0 * l - 1.0) * z;
            R[l][m] = (c1 * a1 - rho2 * a2) * den;
            for (int a = 0; a < 3; ++a) {
                const cplx g1 = dR[l - 1][m][a];
                const cplx g2 = l - 2 >= m ? dR[l - 2][m][a] : cplx(0, 0);
                const double dz = a == 2 ? 1.0 : 0.0;
                const double drho2 = 2.0 * d[a];
                dR[l][m][a] = ((2.0 * l - 1.0) * (dz * a1 + z * g1) - (drho2 * a2 + rho2 * g2)) * den;
            }
        }
    }
}

// Adds the contribution of one quadrature node (position x, weighted normal
// nw) to the moments N (entries for 1 <= l <= L) about centre c.
inline void mpole_add_node(const double x[3], const double nw[3], const double c[3], int L, cplx *N)
{
    cplx R[kMaxLTail3 + 1][kMaxLTail3 + 1], dR[kMaxLTail3 + 1][kMaxLTail3 + 1][3];
    const double d[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
    regular_harmonics(d, L, R, dR);
    for (int l = 1; l <= L; ++l)
        for (int m = 0; m <= l; ++m) {
            cplx s(0, 0);
            for (int a = 0; a < 3; ++a) s += nw[a] * std::conj(dR[l][m][a]);
            N[mp_index(l, m)] -= s;
        }
}

// Adds to Ndst the moments Nsrc (about c_src) translated to c_dst.
inline void mpole_translate(const cplx *Nsrc, const double c_src[3], const double c_dst[3], int L, cplx *Ndst)
{
    cplx R[kMaxLTail3 + 1][kMaxLTail3 + 1], dR[kMaxLTail3 + 1][kMaxLTail3 + 1][3];
    const double d[3] = {c_src[0] - c_dst[0], c_src[1] - c_dst[1], c_src[2] - c_dst[2]};
    regular_harmonics(d, L, R, dR);
    auto getR = [&](int n, int mu) -> cplx {
        if (n < 0 || mu > n || -mu > n) return cplx(0, 0);
        if (mu >= 0) return R[n][mu];
        return (mu & 1 ? -1.0 : 1.0) * std::conj(R[n][-mu]);
    };
    auto getN = [&](int j, int k) -> cplx {
        if (k >= 0) return Nsrc[mp_index(j, k)];
        return (k & 1 ? -1.0 : 1.0) * std::conj(Nsrc[mp_index(j, -k)]);
    };
    for (int l = 1; l <= L; ++l)
        for (int m = 0; m <= l; ++m) {
            cplx s(0, 0);
            for (int j = 1; j <= l; ++j)
                for (int k = -j; k <= j; ++k) {
                    const cplx r = getR(l - j, m - k);
                    if (r != cplx(0, 0)) s += std::conj(r) * getN(j, k);
                }
            Ndst[mp_index(l, m)] += s;
        }
}

// The cluster's solid-angle terms of each degree at offset d = q - c from
// its centre: T[l - 1] = I_l^0 N_l^0 + 2 sum_{m >= 1} Re(I_l^m N_l^m) for
// l = 1 .. L, with the irregular harmonics I_l^m(d) of the device's
// recurrences (unscaled moments N).
inline void mpole_degree_terms(const double d[3], const cplx *N, int L, double *T)
{
    const double inv2 = 1.0 / (d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int l = 1; l <= L; ++l) T[l - 1] = 0.0;
    cplx mm(std::sqrt(inv2), 0.0);
    for (int m = 0; m <= L; ++m) {
        if (m > 0) mm = mm * cplx(d[0], d[1]) * ((2.0 * m - 1.0) * inv2);
        const double wgt = m == 0 ? 1.0 : 2.0;
        cplx prev(0, 0), cur = mm;
        for (int l = m; l <= L; ++l) {
            if (l > m) {
                const double a = (2.0 * l - 1.0) * d[2] * inv2;
                const double b = (double)((l + m - 1) * (l - m - 1)) * inv2;
                const cplx nx = a * cur - b * prev;
                prev = cur;
                cur = nx;
            }
            if (l >= 1) {
                const cplx v = N[mp_index(l, m)];
                T[l - 1] += wgt * (cur.real() * v.real() - cur.imag() * v.imag());
            }
        }
    }
}

}  // namespace gwn
