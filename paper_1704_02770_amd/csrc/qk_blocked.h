// Block tables of the blocked matrix-free H x (Sec. 3 "Hamiltonian matrix
// construction", Eq. (1)), shared by the one-pass kernels (qk_blocked.hip)
// and the two-pass high/low split (qk_split.hip).
//
// A state s splits into its high bits a = s >> llo and its low bits
// b = s & (2^llo - 1).  The sorted basis lists all states with the same a
// contiguously (a "block"); the row of s inside its block is the rank of b
// among the low states of its popcount.
#pragma once

#include "qk_device.h"

namespace qk {

constexpr int kMaxHi = 24;   // row shifts per block entry (high bonds <= 23, zero-padded to a multiple of 4)

// One block of the sorted basis.  Everything the rows of the block share is
// precomputed here and read with scalar loads.
struct BlkEntry {
  uint32_t a;               // high bits
  uint32_t off;             // first row
  uint32_t offw;            // first row of the ring-partner block (high bits with the top bit flipped)
  uint32_t nact;            // number of active high bonds (their two bits differ)
  double dconst;            // block part of the diagonal (high fields, high zz bonds, constants)
  int32_t delta[kMaxHi];    // row shift of each active high bond, then zeros
  uint32_t pad[2];
};
static_assert(sizeof(BlkEntry) == 128, "block entry is two scalar cache lines");

// Block part of the diagonal of every entry from the fields (device, on s).
qk_status launch_block_consts(BlkEntry* blk, int nblk, int llo, int lhi, double zz0, double hhalf, double jz,
                              const double* fields, hipStream_t s);

}  // namespace qk
