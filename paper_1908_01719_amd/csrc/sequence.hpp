// Temporal gradient profiles f(t) and their integral F(t) on the time grid
// (Sec. 2, eq. pgse and eq. b_value; Sec. 3, "General diffusion-encoding
// sequence"; Sec. 4, PGSE / double PGSE / cos-OGSE / sin-OGSE / trapezoidal /
// double trapezoidal profiles).
#pragma once

#include <cstdint>
#include <vector>

namespace dmri {

// What the time loop needs from a sequence, on the grid t^n = n dt:
//   F[n]      = F(t^n), n = 0..N                (transformed form)
//   f_start[n] = f(t^{n-1}+), f_end[n] = f(t^n-), n = 1..N (U-form; index 0 unused)
//   int_F2    = int_0^T F^2 (b = G^2 int_F2)
struct SequenceTables {
    double dt = 0, theta = 0.5;
    int n_steps = 0;
    std::vector<double> F, f_start, f_end;
    bool has_f = false;   // f tables present (a table sequence may omit them)
    double int_F2 = 0;
};

// Builds the tables of a named profile (kind as in include/dmri.h) with its
// parameters; throws Error(DMRI_E_INVALID) on bad parameters or when a
// breakpoint of f or the echo time is not a multiple of dt.
SequenceTables make_sequence(int32_t kind, const double* params, int32_t n_params, double dt,
                             double theta);

}  // namespace dmri
