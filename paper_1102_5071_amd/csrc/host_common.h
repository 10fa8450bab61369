// Host-side input handling shared by the single-trajectory and batched
// entry points: staging of caller matrices, CSR validation, drive copies.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "cfet.h"
#include "cfet_internal.h"

namespace cfet {

// A caller CSR viewed on the host (device arrays are copied into the buffers).
struct HostCSR {
  int64_t n, nnz;
  const int64_t* rp;
  const int32_t* col;
  const double* val;
  std::vector<int64_t> rp_buf;
  std::vector<int32_t> col_buf;
  std::vector<double> val_buf;
};

// True if p is device (or managed) memory; false for plain host memory.
bool is_device_ptr(const void* p);

// Each returns CFET_OK or an error code and sets err to a message.
int load_csr(std::string& err, const cfet_csr* m, const char* name, HostCSR* h);
int validate_csr(std::string& err, const HostCSR& h, const char* name);
int check_hermitian(std::string& err, const HostCSR& h, const char* name);
int copy_drive(std::string& err, const cfet_drive& d, DriveSpec* out);

// Reverse Cuthill-McKee order of the union of the matrices' patterns (row
// adjacency; the operators are Hermitian, so rows and columns carry the same
// pattern): breadth-first levels from a pseudo-peripheral row of each
// connected part, neighbours taken by increasing degree, the whole sequence
// reversed.  Returns order[new] = old.
std::vector<int32_t> rcm_order(const std::vector<HostCSR>& mats, int64_t n);

// Entries (over all matrices) whose row and column fall in different blocks
// of `per` consecutive rows, with rows relabelled old -> inv[old] (null: as
// given).
int64_t cross_block_entries(const std::vector<HostCSR>& mats, int64_t n, int64_t per,
                            const int32_t* inv);

}  // namespace cfet
