// grid.hpp -- the fixed table grid of libcmc.
//
// The paper tabulates the ion-frame cross sections (Sec. III.A) without
// fixing a grid; the grid below is part of the definition of the tabulated
// method.  Every table row covers an abscissa t in [0, 1] split into
// kPanels panels, each integrated with kGauss-point Gauss-Legendre; rows
// store the total, the photon-energy moment (Bremsstrahlung) and the
// normalised cumulative distribution at the panel edges.
#pragma once

namespace cmc {
namespace grid {

constexpr int kPanels = 64;            // CDF panels per row
constexpr int kRow = kPanels + 1;      // CDF values per row
constexpr int kGauss = 8;              // Gauss-Legendre points per panel
constexpr double kCut = 1.0e-7;        // photon energy cut k/(g1-1) = 10^-n, n = 7
constexpr double kTminEv = 1000.0;     // Bremsstrahlung only above 1 keV kinetic
constexpr double kTop = 2.0e4;         // top of every energy axis (10 GeV)
constexpr double kMec2Ev = 510998.95;

// non-relativistic Bremsstrahlung: u = ln(g - 1) in [ln(1 keV/mc^2), 0]
constexpr int kNR = 23;
// moderately relativistic: u = ln g in [ln 2, ln 100]
constexpr int kRel = 56;
// ultra-relativistic: u = ln g in [ln 100, ln 2e4]
constexpr int kUR = 75;
// Bethe-Heitler: u = ln(k - 2) in [ln 1e-6, ln(2e4 - 2)]
constexpr int kBH = 166;
constexpr double kBHx0 = 1.0e-6;
// Trident pair energy: u = ln g1 in [ln 3, ln 2e4]
constexpr int kTri = 124;
// Trident positron split: u = ln g_pair in [ln 4, ln 2e4]
constexpr int kSplit = 120;
// screening length axis: ln L in [ln 10, ln 1e6]
constexpr int kL = 81;
constexpr double kLmin = 10.0, kLmax = 1.0e6;
// Debye fraction axis of the non-relativistic segment: eta_D in [0, 1]
constexpr int kEta = 17;

// table arrays in export order
enum Which { kSigR = 0, kSkR, kCdfR, kSigU, kSkU, kCdfU, kSigN, kSkN, kCdfN,
             kSigB, kCdfB, kCdfT, kCdfS, kNumArrays };

constexpr long long kCount[kNumArrays] = {
    (long long)kRel * kL, (long long)kRel * kL, (long long)kRel * kL * kRow,
    (long long)kUR * kL, (long long)kUR * kL, (long long)kUR * kL * kRow,
    (long long)kNR * kEta * kL, (long long)kNR * kEta * kL, (long long)kNR * kEta * kL * kRow,
    (long long)kBH * kL, (long long)kBH * kL * kRow,
    (long long)kTri * kRow, (long long)kSplit * kRow};

}  // namespace grid
}  // namespace cmc
