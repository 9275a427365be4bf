// Table of the compiled processes; the entries are written by the process
// compiler (paper_2303_18244_amd.codegen) next to the generated kernels.
#pragma once
#include "me_kernel.h"

namespace mgme {

enum ProcKind { KIND_EE = 0, KIND_QCD = 1 };

struct ProcEntry {
  const char* name;
  int n_ext;
  int pdg[8];
  int kind;
  int n_diagrams, n_terms, n_colour, n_currents, n_amps;
  int gs_power;          // power of gs common to every diagram, squared
  int spin_colour_avg;   // initial-state spin and colour average denominator
  int ident;             // final-state identical-particle factor
  long long cden;        // colour-matrix common denominator
  double flops_per_hel;
  double flops_per_event;
  LaunchFn launch;
  const long long* colour_num;  // n_colour^2 numerators
  const int* basis;             // n_colour x n_gluons legs
  int n_gluons;
  int staged;                   // colour-flow vector staged in device memory (many flows)
  int n_overflow;               // staged: overflow slots per (event, helicity)
  unsigned long long kernel_hash;  // FNV-1a hash of the process's generated kernel sources
};

// Device workspace one mgme_matrix_element call takes from the stream-ordered
// allocator (mirrors the sub-batching of the launchers).
long long workspace_bytes(const ProcEntry& e, int nhel, long long nevt, int prec);

extern const ProcEntry kProcesses[];
extern const int kNumProcesses;

}  // namespace mgme
