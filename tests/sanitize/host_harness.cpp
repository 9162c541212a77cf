// Host harness for the library's host-only parsers and table builders,
// built with the address and undefined-behaviour sanitizers (test
// infrastructure): the tune-file JSON reader over given and mutated
// documents, and the twiddle-table builders over every radix plan and
// four-step split shape.
//   host_harness parse FILE...     one line per file: "ok" or "fail"
//   host_harness fuzz SEED ITERS FILE   random byte mutations of FILE
//   host_harness twiddles          table sizes and unit modulus
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "json_lite.hpp"
#include "twiddles.hpp"

using namespace stockfft;

static std::string slurp(const char* path) {
  std::ifstream f(path, std::ios::binary);
  std::stringstream ss;
  ss << f.rdbuf();
  return ss.str();
}

static bool parses(const std::string& text) {
  json::Value v;
  return json::Parser(text).parse(&v);
}

static int twiddles() {
  int bad = 0;
  const int radices[] = {2, 4, 8, 16};
  // every plan of 1 to 5 passes with a product in [2, 16384]
  std::vector<int> plan;
  std::vector<float> out;
  long plans = 0;
  auto visit = [&](auto&& self, int64_t prod) -> void {
    if (!plan.empty()) {
      for (int paired = 0; paired < 2; ++paired) {
        stockham_twiddles(plan.data(), (int)plan.size(), paired == 1, out);
        int64_t want = 0, ns = plan[0], pads = 0;
        for (size_t p = 1; p < plan.size(); ++p) {
          const bool pr = paired && plan[p] >= 4;
          want += (pr ? plan[p] : plan[p] - 1) * ns;
          pads += pr ? ns : 0;
          ns *= plan[p];
        }
        if ((int64_t)out.size() != 2 * want) ++bad;
        int64_t zeros = 0;
        for (size_t i = 0; i + 1 < out.size(); i += 2) {
          const double m = (double)out[i] * out[i] + (double)out[i + 1] * out[i + 1];
          if (m == 0.0)
            ++zeros;
          else if (!(std::fabs(m - 1.0) < 1e-6))
            ++bad;
        }
        if (zeros != pads) ++bad;
        ++plans;
      }
    }
    if (plan.size() == 5) return;
    for (int r : radices) {
      if (prod * r > 16384) continue;
      plan.push_back(r);
      self(self, prod * r);
      plan.pop_back();
    }
  };
  visit(visit, 1);
  long splits = 0;
  for (int64_t n1 = 2; n1 <= 1024; n1 *= 2)
    for (int64_t n2 = 256; n2 <= 16384; n2 *= 2) {
      if (n1 * n2 > (int64_t(1) << 20)) continue;
      for (int tl = 0; tl < 2; ++tl) {
        if (!tl && n1 > 16) continue;
        four_step_twiddles(n1, n2, tl == 1, out);
        const int64_t N = n1 * n2;
        const int s = ilog2_i64(N) / 2;
        const int64_t want = tl ? (int64_t(1) << s) + (N >> s) + n1 : (n1 - 1) * n2;
        if ((int64_t)out.size() != 2 * want) ++bad;
        ++splits;
      }
    }
  std::printf("twiddles: %ld plans, %ld splits, %d bad\n", plans, splits, bad);
  return bad ? 1 : 0;
}

int main(int argc, char** argv) {
  if (argc < 2) return 2;
  const std::string mode = argv[1];
  if (mode == "parse") {
    for (int i = 2; i < argc; ++i) std::printf("%s\n", parses(slurp(argv[i])) ? "ok" : "fail");
    return 0;
  }
  if (mode == "fuzz" && argc == 5) {
    unsigned long long s = std::strtoull(argv[2], nullptr, 10);
    const long iters = std::strtol(argv[3], nullptr, 10);
    const std::string base = slurp(argv[4]);
    auto rnd = [&s]() {
      s = s * 6364136223846793005ULL + 1442695040888963407ULL;
      return (unsigned)(s >> 33);
    };
    const char alphabet[] = "{}[]\",:\\u0123456789eE+-.ntrfaslx \n";
    long accepted = 0;
    for (long it = 0; it < iters; ++it) {
      std::string t = base;
      const int edits = 1 + (int)(rnd() % 8);
      for (int e = 0; e < edits && !t.empty(); ++e) {
        const size_t at = rnd() % t.size();
        switch (rnd() % 4) {
          case 0: t[at] = alphabet[rnd() % (sizeof alphabet - 1)]; break;
          case 1: t.erase(at, 1 + rnd() % 4); break;
          case 2: t.insert(at, 1, alphabet[rnd() % (sizeof alphabet - 1)]); break;
          default: t.resize(at); break;
        }
      }
      accepted += parses(t) ? 1 : 0;
    }
    std::printf("fuzz: %ld of %ld mutations parsed\n", accepted, iters);
    return 0;
  }
  if (mode == "twiddles") return twiddles();
  return 2;
}
