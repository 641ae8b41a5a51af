// Per-order constant tables (see tables.hip).
#pragma once
#include <string>
#include <vector>
#include "common.h"

namespace fmm {
// Device tables for order p on the current device, built on first use and kept
// for the life of the process.  host_copy (optional) receives the struct with
// the same device pointers.  Returns nullptr and sets err on failure.
const OrderTables *get_order_tables(int p, const OrderTables **host_copy, std::string &err);
int host_order_tables(int p, int which, std::vector<double> &out);
// Rotation-based M2L factors (rotation.hip): 0 F, 1 B, 2 A, 3 A index per class
int host_rotation_tables(int p, int which, std::vector<double> &out);
// Taylor coefficients a_g(x) of 1/|x| (|g| <= maxdeg, g_z <= maxz) in long
// double, by mono_index of order maxdeg (the recurrence of tables.hip)
void inv_r_taylor(const long double x[3], int maxdeg, int maxz, std::vector<long double> &a);
} // namespace fmm
