// Physical constants (CODATA 2018, SI) and derived quantities used by the
// library.  Paper Sec. 2: Schwinger field E_s = m_e^2 c^3 / (q_e hbar); the
// total rates of Sec. 2.1 / 2.2 carry the prefactor alpha m_e c^2 / hbar.
#pragma once

namespace qedmi {

constexpr double kMe = 9.1093837015e-31;      // electron mass, kg
constexpr double kC = 299792458.0;            // speed of light, m/s
constexpr double kQe = 1.602176634e-19;       // elementary charge, C
constexpr double kHbar = 1.054571817e-34;     // reduced Planck constant, J s
constexpr double kAlpha = 7.2973525693e-3;    // fine-structure constant

constexpr double kEs = kMe * kMe * kC * kC * kC / (kQe * kHbar);   // V/m
constexpr double kInvEs = 1.0 / kEs;
constexpr double kCOverEs = kC / kEs;                               // (m/s) / (V/m)
constexpr double kRateR0 = kAlpha * kMe * kC * kC / kHbar;          // 1/s

constexpr double kPi = 3.14159265358979323846;

}  // namespace qedmi
