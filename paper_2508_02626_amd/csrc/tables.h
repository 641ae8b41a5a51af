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
} // namespace fmm
