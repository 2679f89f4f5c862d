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
constexpr double kDelta = 0.05;                  // |u - x| split of the resonant piece
constexpr int kRows = 64;                        // rows in |x|
constexpr int kRowsLin = 48;                     // uniform rows on [0, 8): step 1/6
constexpr double kXMax = 300.0;                  // last logarithmic row
constexpr int kMassN = 1024;                     // piece probabilities on x = i/128
constexpr int kQS = 32;                          // quantile nodes, resonant piece
constexpr int kQL = 128;                         // quantile nodes, left piece
constexpr int kQR = 64;                          // quantile nodes, right piece

// ---- one line's table block (floats), 16-byte aligned offsets -------------
constexpr int kOffVoigtCore = 0;
constexpr int kOffVoigtWing = kOffVoigtCore + 4 * kVoigtCoreN;          // 2048
constexpr int kOffMass = kOffVoigtWing + 4 * kVoigtWingN;               // 2560
constexpr int kOffSpike = kOffMass + 2 * (kMassN + 1) + 2;              // 4612
constexpr int kOffLeft = kOffSpike + kRows * kQS;                       // 6660
constexpr int kOffRight = kOffLeft + kRows * kQL;                       // 14852
constexpr int kTabFloats = kOffRight + kRows * kQR;                     // 18948
static_assert(kOffMass % 4 == 0 && kOffSpike % 4 == 0 && kOffLeft % 4 == 0 &&
              kOffRight % 4 == 0 && kTabFloats % 4 == 0, "16-byte aligned blocks");

// host side (krt_tables.cpp)
double row_x(int j);
void build_line_tables(double a, std::vector<float> &tab);
double table_voigt(const std::vector<float> &tab, double x);
double voigt_reference(double a, double x);

}  // namespace krt
