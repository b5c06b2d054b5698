// Lattice constants of the model (Sec. 3(d) listing): honeycomb a = 0.24595 nm
// with a1 = (a, 0), a2 = (a/2, a sqrt(3)/2), A at (0, -a_cc/2) and B at
// (0, +a_cc/2), a_cc = 0.142 nm; square lattice a = 0.24595 nm.
#pragma once

namespace kpm {
constexpr double kAHc = 0.24595, kAccHc = 0.142, kASq = 0.24595;
}  // namespace kpm
