// krt_internal.h -- layout constants shared by the table builder (host) and the
// transport kernels (device) of libkrt.  Not part of the C ABI.
#pragma once
#include <vector>

namespace krt {

// ---- Voigt profile tables (cubic per interval, 4 floats each) -------------
constexpr int kVoigtCoreN = 512;                 // intervals on [0, 8)
constexpr double kVoigtCoreH = 1.0 / 64.0;       // interval width in x
constexpr int kVoigtWingN = 128;                 // intervals in w = 8/|x| on (0, 1]
constexpr double kXLin = 8.0;                    // core/wing split, linear-row limit

// ---- atom-velocity sampler -----------------------------------------------
// pieces of p(u | x), x >= 0, s = |u - x|:
//   S  : |u - x| < DELTA            variable t = theta/theta_DELTA, u = x + a tan(theta)
//   L1 : x - SMID < u <= x - DELTA  variable l = ln(s/DELTA)
//   L2 : u <= x - SMID              variable u itself (the thermal bump)
//   R  : u >= x + DELTA             variable l = ln(s/DELTA)
// with SMID = max(x/2, 2 DELTA).
constexpr double kDelta = 0.05;
constexpr int kRows = 64;                        // rows in |x|
constexpr int kRowsLin = 48;                     // uniform rows on [0, 8): step 1/6
constexpr double kXMax = 300.0;                  // last logarithmic row
constexpr int kMassN = 512;                      // piece probabilities on x = i/64
constexpr int kQS = 32;                          // quantile nodes per row, S
constexpr int kQL1 = 64;                         // L1
constexpr int kQL2 = 64;                         // L2
constexpr int kQR = 64;                          // R

// ---- one line's table block (floats), 16-byte aligned offsets -------------
constexpr int kOffVoigtCore = 0;
constexpr int kOffVoigtWing = kOffVoigtCore + 4 * kVoigtCoreN;          // 2048
constexpr int kOffMass = kOffVoigtWing + 4 * kVoigtWingN;               // 2560: float4 (cS, cL1, cL2, 1) per node
constexpr int kOffSpike = kOffMass + 4 * (kMassN + 1);                  // 4612
constexpr int kOffL1 = kOffSpike + kRows * kQS;                         // 6660
constexpr int kOffL2 = kOffL1 + kRows * kQL1;                           // 10756
constexpr int kOffRight = kOffL2 + kRows * kQL2;                        // 14852
constexpr int kTabFloats = kOffRight + kRows * kQR;                     // 18948
constexpr int kVoigtFloats = kOffMass;                                  // the Voigt part: 2560
static_assert(kOffMass % 4 == 0 && kOffSpike % 4 == 0 && kOffL1 % 4 == 0 && kOffL2 % 4 == 0 &&
              kOffRight % 4 == 0 && kTabFloats % 4 == 0, "16-byte aligned blocks");
static_assert(kQL1 == kQL2 && kQL2 == kQR, "one node count for the wing pieces");
static_assert(kTabFloats * 4 <= 80 * 1024, "two workgroups' tables fit the 160 KiB LDS of a CU");

// host side (krt_tables.cpp)
double row_x(int j);
void build_line_tables(double a, std::vector<float> &tab);
// the two parts of one table block: the Voigt lookup (floats [0, kVoigtFloats))
// and the sampler (mass table and quantile rows), each into a block of kTabFloats
void build_voigt_block(double a, float *tab);
void build_sampler_block(double a, float *tab);
double table_voigt(const std::vector<float> &tab, double x);
double voigt_reference(double a, double x);

}  // namespace krt
