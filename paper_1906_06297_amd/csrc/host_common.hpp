// Host-side helpers shared by the C ABI translation units (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ising.h"
#include "ising_device.hpp"

namespace ising {
namespace host {

// Records the message for ising_last_error() and returns `code`.
int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
int ok();
const char *last_error();

// Largest supported size: chunk indices must fit the 32-bit counter word.
constexpr int64_t kMaxL = 741454; // floor(sqrt(128 * (2^32 - 1)))

// Argument checks shared by the entry points (each records the message and
// returns an ISING_E_* code, or ISING_OK).
int check_L(int64_t L);
int check_lattice(const ising_lattice *lat);
int check_temperature(double beta, double J);

// T[a] = 2^32 for dE <= 0, floor(exp(-beta dE) 2^32) otherwise; dE = 4J(a-2).
void threshold_table(double beta, double J, uint64_t T[5]);

// The two classes with dE > 0 under the Metropolis rule and how each is decided.
Metro2 metro2_params(double beta, double J);

} // namespace host
} // namespace ising
