// Reader for LHAPDF6 data files (the set folders the paper loads directly,
// section 2): a member file in the "lhagrid1" layout and the alpha_s knots of
// a set's .info metadata.  Host code only; the arrays it produces are those
// pdf_load_grid / pdf_load_alphas take (Q knots squared in FP64).
//
// Member file layout:
//   a header of "key: value" lines, ended by a line "---";
//   then one block per sub-grid, each ended by a line "---":
//     line 1: the x knots, line 2: the Q knots, line 3: the flavour ids,
//     then nx*nq lines of one value per flavour (x*f), the Q index running
//     fastest (x-major, the order pdf_load_grid takes).
// .info: YAML; the keys AlphaS_Qs and AlphaS_Vals hold flow lists [a, b, ...]
// (possibly over several lines) of Q knots (repeated at flavour thresholds)
// and alpha_s values.
#include <cerrno>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "pdfmi.h"

namespace pdfmi {
int report_error(int code, const char* msg);
}

namespace {

using pdfmi::report_error;

int io_fail(int code, const std::string& msg) { return report_error(code, msg.c_str()); }

bool read_file(const char* path, std::string& text) {
  std::ifstream f(path, std::ios::binary);
  if (!f) return false;
  std::ostringstream ss;
  ss << f.rdbuf();
  text = ss.str();
  return true;
}

// Lines without their end-of-line characters ("\n" or "\r\n").
std::vector<std::string> split_lines(const std::string& text) {
  std::vector<std::string> lines;
  size_t b = 0;
  while (b <= text.size()) {
    size_t e = text.find('\n', b);
    if (e == std::string::npos) e = text.size();
    std::string l = text.substr(b, e - b);
    if (!l.empty() && l.back() == '\r') l.pop_back();
    lines.push_back(l);
    b = e + 1;
  }
  return lines;
}

std::string trim(const std::string& s) {
  size_t b = s.find_first_not_of(" \t"), e = s.find_last_not_of(" \t");
  return b == std::string::npos ? std::string() : s.substr(b, e - b + 1);
}

bool is_separator(const std::string& l) { return trim(l) == "---"; }

// Whitespace-separated numbers of one line; false on any token that is not a number.
bool parse_doubles(const std::string& l, std::vector<double>& out) {
  out.clear();
  const char* p = l.c_str();
  for (;;) {
    while (*p == ' ' || *p == '\t') ++p;
    if (!*p) return true;
    char* end = nullptr;
    errno = 0;
    const double v = std::strtod(p, &end);
    if (end == p || (*end && *end != ' ' && *end != '\t')) return false;
    out.push_back(v);
    p = end;
  }
}

bool parse_ints(const std::string& l, std::vector<int32_t>& out) {
  std::vector<double> d;
  if (!parse_doubles(l, d)) return false;
  out.clear();
  for (double v : d) {
    if (v != (double)(int32_t)v) return false;
    out.push_back((int32_t)v);
  }
  return true;
}

struct Parsed {
  std::vector<int32_t> shape;  // [K][2]
  std::vector<int32_t> pids;
  std::vector<double> knots;   // per sub-grid: x knots, then Q^2 knots
  std::vector<double> values;  // per sub-grid: [ix][iq][flavour]
};

int parse_member(const char* path, Parsed& P) {
  if (!path) return io_fail(PDF_ERR_ARG, "null path");
  std::string text;
  if (!read_file(path, text)) return io_fail(PDF_ERR_ARG, std::string("cannot read ") + path);
  const std::vector<std::string> lines = split_lines(text);
  size_t i = 0;
  // header: "key: value" lines up to the first separator; the format key must name lhagrid1
  bool fmt_ok = true;
  for (; i < lines.size() && !is_separator(lines[i]); ++i) {
    const std::string l = trim(lines[i]);
    if (l.empty()) continue;
    if (l.find(':') == std::string::npos)
      return io_fail(PDF_ERR_GRID, std::string(path) + ": header line " + std::to_string(i + 1) +
                                       " is not 'key: value' (missing '---' after the header?)");
    if (l.rfind("Format:", 0) == 0 && trim(l.substr(7)) != "lhagrid1") fmt_ok = false;
  }
  if (!fmt_ok) return io_fail(PDF_ERR_GRID, std::string(path) + ": not an lhagrid1 member file");
  if (i == lines.size()) return io_fail(PDF_ERR_GRID, std::string(path) + ": no '---' after the header");
  ++i;
  std::vector<double> row;
  for (int k = 0;; ++k) {
    while (i < lines.size() && trim(lines[i]).empty()) ++i;  // trailing blank lines
    if (i == lines.size()) break;
    const std::string where = std::string(path) + ": sub-grid " + std::to_string(k);
    if (i + 3 > lines.size()) return io_fail(PDF_ERR_GRID, where + ": truncated block header");
    std::vector<double> xk, qk;
    std::vector<int32_t> ids;
    if (!parse_doubles(lines[i], xk) || !parse_doubles(lines[i + 1], qk) || !parse_ints(lines[i + 2], ids))
      return io_fail(PDF_ERR_GRID, where + ": malformed knot or flavour line");
    if (xk.size() < 2 || qk.size() < 2 || ids.empty())
      return io_fail(PDF_ERR_GRID, where + ": needs >= 2 x knots, >= 2 Q knots and >= 1 flavour");
    if (k == 0) {
      P.pids = ids;
    } else if (ids != P.pids) {
      return io_fail(PDF_ERR_GRID, where + ": flavour list differs from sub-grid 0");
    }
    i += 3;
    const size_t nrow = xk.size() * qk.size();
    for (size_t r = 0; r < nrow; ++r, ++i) {
      if (i >= lines.size() || is_separator(lines[i]))
        return io_fail(PDF_ERR_GRID, where + ": fewer value lines than nx*nq");
      if (!parse_doubles(lines[i], row) || row.size() != ids.size())
        return io_fail(PDF_ERR_GRID, where + ": value line " + std::to_string(r) + " does not hold one number per flavour");
      P.values.insert(P.values.end(), row.begin(), row.end());
    }
    if (i >= lines.size() || !is_separator(lines[i]))
      return io_fail(PDF_ERR_GRID, where + ": block not ended by '---' after nx*nq value lines");
    ++i;
    P.shape.push_back((int32_t)xk.size());
    P.shape.push_back((int32_t)qk.size());
    P.knots.insert(P.knots.end(), xk.begin(), xk.end());
    for (double q : qk) P.knots.push_back(q * q);
  }
  if (P.shape.empty()) return io_fail(PDF_ERR_GRID, std::string(path) + ": no sub-grid blocks");
  return PDF_OK;
}

// The flow list after "key:" in a YAML text, possibly spanning lines.
int yaml_list(const std::string& text, const char* key, std::vector<double>& out, const char* path) {
  const std::vector<std::string> lines = split_lines(text);
  const std::string k = std::string(key) + ":";
  for (size_t i = 0; i < lines.size(); ++i) {
    const std::string l = trim(lines[i]);
    if (l.rfind(k, 0) != 0) continue;
    std::string acc = l.substr(k.size());
    size_t j = i;
    while (acc.find(']') == std::string::npos && ++j < lines.size()) acc += " " + lines[j];
    const size_t b = acc.find('['), e = acc.find(']');
    if (b == std::string::npos || e == std::string::npos || e < b)
      return io_fail(PDF_ERR_GRID, std::string(path) + ": " + key + " is not a [..] list");
    std::string body = acc.substr(b + 1, e - b - 1);
    for (char& c : body)
      if (c == ',') c = ' ';
    if (!parse_doubles(body, out) || out.empty())
      return io_fail(PDF_ERR_GRID, std::string(path) + ": " + key + " holds a non-number");
    return PDF_OK;
  }
  return io_fail(PDF_ERR_GRID, std::string(path) + ": no " + key + " entry");
}

int parse_alphas(const char* path, std::vector<double>& q2, std::vector<double>& as) {
  if (!path) return io_fail(PDF_ERR_ARG, "null path");
  std::string text;
  if (!read_file(path, text)) return io_fail(PDF_ERR_ARG, std::string("cannot read ") + path);
  std::vector<double> qs;
  int rc = yaml_list(text, "AlphaS_Qs", qs, path);
  if (rc != PDF_OK) return rc;
  if ((rc = yaml_list(text, "AlphaS_Vals", as, path)) != PDF_OK) return rc;
  if (qs.size() != as.size())
    return io_fail(PDF_ERR_GRID, std::string(path) + ": AlphaS_Qs and AlphaS_Vals differ in length");
  q2.clear();
  for (double q : qs) q2.push_back(q * q);
  return PDF_OK;
}

}  // namespace

extern "C" int pdf_lhapdf_read(const char* path, int64_t* sizes, int32_t* shape, int32_t* pids, double* knots,
                               double* values) {
  if (!sizes) return io_fail(PDF_ERR_ARG, "null sizes");
  Parsed P;
  const int rc = parse_member(path, P);
  if (rc != PDF_OK) return rc;
  sizes[0] = (int64_t)P.shape.size() / 2;
  sizes[1] = (int64_t)P.pids.size();
  sizes[2] = (int64_t)P.knots.size();
  sizes[3] = (int64_t)P.values.size();
  if (!shape && !pids && !knots && !values) return PDF_OK;
  if (!shape || !pids || !knots || !values) return io_fail(PDF_ERR_ARG, "pass all four arrays or none");
  std::memcpy(shape, P.shape.data(), P.shape.size() * sizeof(int32_t));
  std::memcpy(pids, P.pids.data(), P.pids.size() * sizeof(int32_t));
  std::memcpy(knots, P.knots.data(), P.knots.size() * sizeof(double));
  std::memcpy(values, P.values.data(), P.values.size() * sizeof(double));
  return PDF_OK;
}

extern "C" int pdf_load_lhapdf(const char* path, int32_t* member_out) {
  Parsed P;
  const int rc = parse_member(path, P);
  if (rc != PDF_OK) return rc;
  return pdf_load_grid((int32_t)(P.shape.size() / 2), P.shape.data(), (int32_t)P.pids.size(), P.pids.data(),
                       P.knots.data(), P.values.data(), member_out);
}

extern "C" int pdf_lhapdf_read_alphas(const char* info_path, int32_t* n_out, double* q2_knots, double* alphas) {
  if (!n_out) return io_fail(PDF_ERR_ARG, "null n_out");
  std::vector<double> q2, as;
  const int rc = parse_alphas(info_path, q2, as);
  if (rc != PDF_OK) return rc;
  *n_out = (int32_t)q2.size();
  if (!q2_knots && !alphas) return PDF_OK;
  if (!q2_knots || !alphas) return io_fail(PDF_ERR_ARG, "pass both arrays or neither");
  std::memcpy(q2_knots, q2.data(), q2.size() * sizeof(double));
  std::memcpy(alphas, as.data(), as.size() * sizeof(double));
  return PDF_OK;
}

extern "C" int pdf_load_lhapdf_alphas(const char* info_path) {
  std::vector<double> q2, as;
  const int rc = parse_alphas(info_path, q2, as);
  if (rc != PDF_OK) return rc;
  return pdf_load_alphas((int32_t)q2.size(), q2.data(), as.data());
}
