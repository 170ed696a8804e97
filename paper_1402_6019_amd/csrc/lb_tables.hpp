// Compile-time tables of the D2Q9 lattice and the two-belt interaction stencil.
//
// D2Q9 (the lattice Boltzmann velocity set, eq. (LB)): c_0..c_8 =
// (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),(-1,-1),(1,-1); weights 4/9, 1/9, 1/36.
//
// Interaction shells (Fig. 1: 24 links in two belts, |c|^2 = 1, 2 | 4, 5, 8).  Default
// isotropic weights with second moment c_s^2 = 1/3, which the bulk equation of state
// (BULK) requires:
//   w (attractive belt, |c|^2 <= 4, sixth-order isotropic) = 4/45, 1/30, 1/360, 0, 0
//   p (both belts, sixth-order isotropic closed by eighth order) =
//     4/63, 4/135, 1/180, 2/945, 1/15120
//   t (A-B repulsion, first belt) = 1/9, 1/36
#pragma once

namespace lb355 {

constexpr int Q = 9;
constexpr int CXS[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int CYS[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int OPPS[Q] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
constexpr double WD2Q9[Q] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

constexpr int NSHELL = 5;  // |c|^2 = 1, 2, 4, 5, 8
constexpr double W_ATTR[NSHELL] = {4.0 / 45.0, 1.0 / 30.0, 1.0 / 360.0, 0.0, 0.0};
constexpr double P_REP[NSHELL] = {4.0 / 63.0, 4.0 / 135.0, 1.0 / 180.0, 2.0 / 945.0, 1.0 / 15120.0};
constexpr double T_CROSS[2] = {1.0 / 9.0, 1.0 / 36.0};

// One link of each +-c pair of the two belts ("half-links"), with its shell index: the force
// sum over 24 links is a sum over these 12 of K(q) c (psi(x + c) - psi(x - c)).  The first
// four form the first belt (|c|^2 = 1, 2) used by the A-B repulsion.
constexpr int NHALF = 12;
constexpr int HX[NHALF] = {1, 0, 1, 1, 2, 0, 2, 1, 1, 2, 2, 2};
constexpr int HY[NHALF] = {0, 1, 1, -1, 0, 2, 1, 2, -2, -1, 2, -2};
constexpr int HQ[NHALF] = {0, 0, 1, 1, 2, 2, 3, 3, 3, 3, 4, 4};

}  // namespace lb355
