// Drives the library's argument checks (paper_1412_8447_amd/csrc/args.cpp) on
// the CPU, one call per input line, for tests/test_host_args.py. Built with the
// address and undefined-behaviour sanitizers; no GPU and no HIP runtime.
//
// Line: <kind> [key=value ...], kind one of id, outs, batched. Every call starts
// from a valid configuration (m = 64, n = 48, lda = 48, k = 5, deterministic,
// FP64 for id / outs, FP32 for batched, all output arrays present) and applies
// the overrides; pointer keys take 0 (NULL) or 1 (present). Output line:
// "<status code> <message or ->".
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <iostream>
#include <sstream>
#include <string>

#include "args.hpp"

using namespace idcur;

namespace {

int dummy[16];

const void* ptr_flag(const std::string& v) { return std::stoll(v) ? static_cast<const void*>(dummy) : nullptr; }

bool set_opt(idcur_opts& o, const std::string& k, const std::string& v) {
  if (k == "k") o.k = std::stoi(v);
  else if (k == "kmax") o.kmax = std::stoi(v);
  else if (k == "tol") o.tol = std::strtod(v.c_str(), nullptr);
  else if (k == "rank_tol") o.rank_tol = std::strtod(v.c_str(), nullptr);
  else if (k == "p") o.p = std::stoi(v);
  else if (k == "q") o.q = std::stoi(v);
  else if (k == "prec") o.prec = std::stoi(v);
  else if (k == "norms") o.norms = std::stoi(v);
  else if (k == "sketch") o.sketch = std::stoi(v);
  else if (k == "u_correct") o.u_correct = std::stoi(v);
  else if (k == "t_reg") o.t_reg = std::strtod(v.c_str(), nullptr);
  else if (k == "t_svd") o.t_svd = std::strtod(v.c_str(), nullptr);
  else if (k == "omega") o.omega = ptr_flag(v);
  else if (k == "srht_rows") o.srht_rows = static_cast<const int32_t*>(ptr_flag(v));
  else if (k == "srht_signs") o.srht_signs = static_cast<const int8_t*>(ptr_flag(v));
  else return false;
  return true;
}

}  // namespace

int main() {
  std::string line;
  while (std::getline(std::cin, line)) {
    if (line.empty()) continue;
    std::istringstream in(line);
    std::string kind;
    in >> kind;
    idcur_opts o;
    std::memset(&o, 0, sizeof o);
    o.p = -1;
    o.k = 5;
    int op = OP_COL, dtype = kind == "batched" ? IDCUR_F32 : IDCUR_F64;
    int64_t m = 64, n = 48, lda = 48;
    int nblk = 8, mmax = 64, nmax = 48;
    bool opts_null = false;
    const void* A = dummy;
    Outs out;
    out.k_out = dummy; out.J = dummy; out.T = dummy; out.ldt = 48;
    out.I = dummy; out.Tr = dummy; out.ldtr = 64;
    out.U = dummy; out.ldu = 48; out.C = dummy; out.ldc = 48; out.R = dummy; out.ldr = 48;
    out.Yt = dummy; out.ldy = 48;
    if (kind == "batched") o.p = 4;
    std::string kv;
    bool bad = false;
    while (in >> kv) {
      const size_t eq = kv.find('=');
      if (eq == std::string::npos) { bad = true; break; }
      const std::string k = kv.substr(0, eq), v = kv.substr(eq + 1);
      if (set_opt(o, k, v)) continue;
      if (k == "op") op = std::stoi(v);
      else if (k == "dtype") dtype = std::stoi(v);
      else if (k == "m") m = std::stoll(v);
      else if (k == "n") n = std::stoll(v);
      else if (k == "lda") lda = std::stoll(v);
      else if (k == "nblk") nblk = std::stoi(v);
      else if (k == "mmax") mmax = std::stoi(v);
      else if (k == "nmax") nmax = std::stoi(v);
      else if (k == "opts") opts_null = std::stoi(v) == 0;
      else if (k == "A") A = ptr_flag(v);
      else if (k == "k_out") out.k_out = std::stoi(v) ? dummy : nullptr;
      else if (k == "J") out.J = std::stoi(v) ? dummy : nullptr;
      else if (k == "I") out.I = std::stoi(v) ? dummy : nullptr;
      else if (k == "T") out.T = std::stoi(v) ? dummy : nullptr;
      else if (k == "Tr") out.Tr = std::stoi(v) ? dummy : nullptr;
      else if (k == "U") out.U = std::stoi(v) ? dummy : nullptr;
      else if (k == "C") out.C = std::stoi(v) ? dummy : nullptr;
      else if (k == "R") out.R = std::stoi(v) ? dummy : nullptr;
      else if (k == "Yt") out.Yt = std::stoi(v) ? dummy : nullptr;
      else if (k == "ldt") out.ldt = std::stoll(v);
      else if (k == "ldtr") out.ldtr = std::stoll(v);
      else if (k == "ldu") out.ldu = std::stoll(v);
      else if (k == "ldc") out.ldc = std::stoll(v);
      else if (k == "ldr") out.ldr = std::stoll(v);
      else if (k == "ldy") out.ldy = std::stoll(v);
      else { bad = true; break; }
    }
    if (bad) {
      std::printf("bad-input -\n");
      std::fflush(stdout);
      continue;
    }
    ArgCheck r{IDCUR_OK, nullptr};
    if (kind == "id") {
      r = check_id_args(op, dtype, m, n, lda, opts_null ? nullptr : &o);
    } else if (kind == "outs") {
      r = check_id_args(op, dtype, m, n, lda, &o);
      if (r.code == IDCUR_OK) r = check_id_outs(op, m, n, A, o, out);
    } else if (kind == "batched") {
      r = check_batched_args(dtype, nblk, mmax, nmax, opts_null ? nullptr : &o, 512, 64);
    } else {
      std::printf("bad-kind -\n");
      std::fflush(stdout);
      continue;
    }
    std::printf("%d %s\n", (int)r.code, r.msg ? r.msg : "-");
    std::fflush(stdout);
  }
  return 0;
}
