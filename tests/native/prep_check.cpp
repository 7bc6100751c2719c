// Host check of the input validation and format conversion of qpg_setup (csrc/host_prep.cpp):
// reads a problem in the C ABI's CSC convention from raw files, runs prepare() and writes the
// converted arrays back, so that the caller can compare them with an independent conversion.
//   prep_check <dir> <n> <m> <rho_vector>
// reads <dir>/{pcp,pri,pv,q,acp,ari,av,l,u}.bin (int32 index arrays, float64 values) and writes
// <dir>/out_{a_ptr,a_col,b_ptr,b_split,b_col,lb,ub,eqrow}.bin (int32 / float64 / uint8) and
// out_{a_val,b_val}.bin; prints "rc <code>" and, on failure, the message.
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <string>
#include <vector>

#include "qpg_internal.hpp"

using namespace qpg;

template <typename T>
static std::vector<T> read_all(const std::string& f) {
  std::ifstream in(f, std::ios::binary | std::ios::ate);
  if (!in) return {};
  const size_t n = (size_t)in.tellg();
  in.seekg(0);
  std::vector<T> v(n / sizeof(T));
  in.read(reinterpret_cast<char*>(v.data()), (std::streamsize)n);
  return v;
}

template <typename V>
static void write_all(const std::string& f, const V& v) {
  std::ofstream out(f, std::ios::binary);
  out.write(reinterpret_cast<const char*>(v.data()), (std::streamsize)(v.size() * sizeof(v[0])));
}

int main(int argc, char** argv) {
  if (argc < 5) return 2;
  const std::string d = argv[1];
  const int n = std::atoi(argv[2]), m = std::atoi(argv[3]), rv = std::atoi(argv[4]);
  const auto pcp = read_all<int32_t>(d + "/pcp.bin"), pri = read_all<int32_t>(d + "/pri.bin");
  const auto acp = read_all<int32_t>(d + "/acp.bin"), ari = read_all<int32_t>(d + "/ari.bin");
  const auto pv = read_all<double>(d + "/pv.bin"), av = read_all<double>(d + "/av.bin");
  const auto q = read_all<double>(d + "/q.bin"), l = read_all<double>(d + "/l.bin"), u = read_all<double>(d + "/u.bin");
  // the declared nnz is the last column pointer, as the binding passes it; an inconsistent
  // colptr is then the library's to reject
  qpg_csc P{n, n, pcp.empty() ? 0 : pcp.back(), pcp.data(), pri.data(), pv.data()};
  qpg_csc A{m, n, acp.empty() ? 0 : acp.back(), acp.data(), ari.data(), av.data()};
  qpg_settings s;
  qpg_default_settings(&s);
  s.rho_vector = rv;
  HostProblem H;
  std::string msg;
  const int rc = prepare(&P, q.data(), &A, m ? l.data() : nullptr, m ? u.data() : nullptr, &s, &H, &msg);
  std::printf("rc %d\n%s\n", rc, msg.c_str());
  if (rc) return 0;
  // the values as the device places them (qpg_solver::place_raw): Ā's through the CSR → CSC
  // index map, B's rows from the full P's rows and A's columns
  std::vector<double> a_val(H.a_src.size()), b_val(H.b_col.size());
  for (size_t k = 0; k < a_val.size(); ++k) {
    if (H.a_src[k] < 0 || H.a_src[k] >= A.nnz) {
      std::printf("a_src out of range\n");
      return 1;
    }
    a_val[k] = H.a_csc_val[H.a_src[k]];
  }
  for (int i = 0; i < n; ++i) {
    const int32_t o = H.b_ptr[i], sp = H.b_split[i];
    if (sp - o != H.p_ptr[i + 1] - H.p_ptr[i] || H.b_ptr[i + 1] - sp != H.a_colptr[i + 1] - H.a_colptr[i]) {
      std::printf("B row %d: part lengths\n", i);
      return 1;
    }
    for (int32_t k = 0; k < sp - o; ++k) b_val[o + k] = H.p_val[H.p_ptr[i] + k];
    for (int32_t k = 0; k < H.b_ptr[i + 1] - sp; ++k) b_val[sp + k] = H.a_csc_val[H.a_colptr[i] + k];
  }
  write_all(d + "/out_a_ptr.bin", H.a_ptr);
  write_all(d + "/out_a_col.bin", H.a_col);
  write_all(d + "/out_a_val.bin", a_val);
  write_all(d + "/out_b_ptr.bin", H.b_ptr);
  write_all(d + "/out_b_split.bin", H.b_split);
  write_all(d + "/out_b_col.bin", H.b_col);
  write_all(d + "/out_b_val.bin", b_val);
  write_all(d + "/out_lb.bin", H.lb);
  write_all(d + "/out_ub.bin", H.ub);
  write_all(d + "/out_eqrow.bin", H.eqrow);
  return 0;
}
