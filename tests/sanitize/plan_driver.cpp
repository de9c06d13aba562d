// plan_driver.cpp -- drives the host planner through its C-ABI in a CPU build
// under AddressSanitizer / UndefinedBehaviorSanitizer (test infrastructure).
// Every case is planned host-only (and its work decomposition checked on the
// host), then planned against the host-memory device of hip_host_stub.cpp
// with each of its device allocations failing in turn: each failure must
// return SPINSUM_ERR_OUT_OF_MEMORY with no plan and no allocation left over,
// and a failed re-tiling must leave a plan that still answers and frees
// everything when destroyed.  LeakSanitizer checks the host side at exit.
// Prints one line per case; exit status 0 when every check held.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <numeric>
#include <string>
#include <vector>

#include "spinsum.h"

extern "C" void stub_fail_alloc_at(long k);
extern "C" long stub_live_allocations(void);
extern "C" long stub_allocations_made(void);

namespace {

int g_fail = 0;

void check(bool ok, const std::string& what) {
  if (!ok) {
    std::printf("FAIL %s\n", what.c_str());
    ++g_fail;
  }
}

struct Case {
  std::string name;
  std::vector<int64_t> shape;
  int gf, d;
  std::vector<std::vector<std::pair<std::vector<int>, double>>> stages;
  unsigned flags;
  spinsum_dtype dtype;
  int inplace;
  std::vector<spinsum_tile_t> tiles;  // re-tilings to try
};

struct Flat {
  std::vector<int> nterms, perms;
  std::vector<double> alpha;
};

Flat flatten(const Case& c) {
  Flat f;
  for (const auto& st : c.stages) {
    f.nterms.push_back((int)st.size());
    for (const auto& t : st) {
      f.perms.insert(f.perms.end(), t.first.begin(), t.first.end());
      f.alpha.push_back(t.second);
    }
  }
  return f;
}

std::vector<std::pair<std::vector<int>, double>> all_perms(int d, unsigned seed) {
  std::vector<int> p(d);
  std::iota(p.begin(), p.end(), 0);
  std::vector<std::pair<std::vector<int>, double>> out;
  unsigned s = seed;
  do {
    s = s * 1103515245u + 12345u;
    out.push_back({p, (double)((int)((s >> 16) % 11) - 2)});
  } while (std::next_permutation(p.begin(), p.end()));
  return out;
}

std::vector<int> P(const char* s) {
  std::vector<int> p;
  for (const char* c = s; *c; ++c) p.push_back(*c - '1');
  return p;
}

spinsum_status make(const Case& c, unsigned flags, spinsum_plan_t* plan) {
  Flat f = flatten(c);
  return spinsum_plan(plan, (int)c.shape.size(), c.shape.data(), c.gf, c.d, (int)f.nterms.size(),
                      f.nterms.data(), f.perms.data(), f.alpha.data(), c.dtype, c.inplace,
                      flags);
}

void run_case(const Case& c) {
  // host-only plan: tables, info, expansion, ownership
  spinsum_plan_t p = nullptr;
  spinsum_status st = make(c, c.flags | SPINSUM_FLAG_HOST_ONLY, &p);
  check(st == SPINSUM_OK && p, c.name + ": host-only plan");
  if (!p) return;
  spinsum_plan_info_t info;
  check(spinsum_plan_get_info(p, &info) == SPINSUM_OK, c.name + ": info");
  int nt = 0;
  std::vector<int> perms(24 * 4);
  std::vector<double> alpha(24);
  check(spinsum_plan_expanded(p, 24, &nt, perms.data(), alpha.data()) == SPINSUM_OK,
        c.name + ": expanded");
  const char* why = nullptr;
  check(spinsum_plan_check_ownership(p, 0, &why) == SPINSUM_OK,
        c.name + ": ownership " + (why ? why : ""));
  for (const spinsum_tile_t& t : c.tiles) {
    spinsum_status s2 = spinsum_plan_set_tile(p, &t);
    if (s2 == SPINSUM_OK) {
      check(spinsum_plan_check_ownership(p, 0, &why) == SPINSUM_OK,
            c.name + ": ownership after set_tile bl=" + std::to_string(t.bl) + " " +
                (why ? why : ""));
    } else {
      check(s2 == SPINSUM_ERR_UNSUPPORTED, c.name + ": set_tile status");
    }
  }
  spinsum_plan_destroy(p);

  // device plan, every allocation failing in turn
  long made = -1;
  for (long k = 1; k <= 64; ++k) {
    stub_fail_alloc_at(k);
    p = nullptr;
    st = make(c, c.flags, &p);
    if (st == SPINSUM_OK) {
      made = stub_allocations_made();
      check(made < k, c.name + ": plan succeeded although allocation " + std::to_string(k) +
                          " failed");
      spinsum_plan_destroy(p);
      check(stub_live_allocations() == 0, c.name + ": leak after destroy");
      break;
    }
    check(st == SPINSUM_ERR_OUT_OF_MEMORY, c.name + ": status " + std::to_string((int)st) +
                                               " at failed allocation " + std::to_string(k));
    check(p == nullptr, c.name + ": plan returned on failure");
    check(stub_live_allocations() == 0,
          c.name + ": leak after failed allocation " + std::to_string(k));
  }
  check(made > 0, c.name + ": never planned");
  // a failed re-tiling keeps a usable plan
  for (const spinsum_tile_t& t : c.tiles) {
    for (long k = 1; k <= 16; ++k) {
      stub_fail_alloc_at(0);
      p = nullptr;
      if (make(c, c.flags, &p) != SPINSUM_OK) {
        check(false, c.name + ": replan");
        break;
      }
      stub_fail_alloc_at(k);
      spinsum_status s2 = spinsum_plan_set_tile(p, &t);
      stub_fail_alloc_at(0);
      check(spinsum_plan_get_info(p, &info) == SPINSUM_OK, c.name + ": info after set_tile");
      spinsum_plan_destroy(p);
      check(stub_live_allocations() == 0, c.name + ": leak after set_tile failure");
      if (s2 != SPINSUM_ERR_OUT_OF_MEMORY) break;
    }
  }
  stub_fail_alloc_at(0);
  std::printf("ok %s (%ld device tables)\n", c.name.c_str(), made);
}

void batched_case(const std::string& name, const std::vector<std::vector<int64_t>>& shapes, int gf,
                  int d, const std::vector<std::pair<std::vector<int>, double>>& terms) {
  std::vector<int> ndims;
  std::vector<const int64_t*> ext;
  for (const auto& s : shapes) {
    ndims.push_back((int)s.size());
    ext.push_back(s.data());
  }
  std::vector<int> nterms{(int)terms.size()}, perms;
  std::vector<double> alpha;
  for (const auto& t : terms) {
    perms.insert(perms.end(), t.first.begin(), t.first.end());
    alpha.push_back(t.second);
  }
  spinsum_plan_t p = nullptr;
  auto mk = [&](unsigned fl) {
    return spinsum_plan_batched(&p, (int)shapes.size(), ndims.data(), ext.data(), gf, d, 1,
                                nterms.data(), perms.data(), alpha.data(), SPINSUM_F64, 1, fl);
  };
  check(mk(SPINSUM_FLAG_HOST_ONLY) == SPINSUM_OK && p, name + ": host-only batched plan");
  if (p) {
    for (int b = 0; b < (int)shapes.size(); ++b) {
      const char* why = nullptr;
      check(spinsum_plan_check_ownership(p, b, &why) == SPINSUM_OK,
            name + ": ownership block " + std::to_string(b) + " " + (why ? why : ""));
    }
    spinsum_plan_destroy(p);
  }
  long made = -1;
  for (long k = 1; k <= 64; ++k) {
    stub_fail_alloc_at(k);
    p = nullptr;
    spinsum_status st = mk(0);
    if (st == SPINSUM_OK) {
      made = stub_allocations_made();
      spinsum_plan_destroy(p);
      check(stub_live_allocations() == 0, name + ": leak after destroy");
      break;
    }
    check(st == SPINSUM_ERR_OUT_OF_MEMORY && p == nullptr, name + ": failure status");
    check(stub_live_allocations() == 0, name + ": leak after failed allocation");
  }
  stub_fail_alloc_at(0);
  check(made > 0, name + ": never planned");
  std::printf("ok %s (%ld device tables)\n", name.c_str(), made);
}

}  // namespace

int main() {
  const auto A3 = std::vector<std::pair<std::vector<int>, double>>{
      {P("123"), 4}, {P("213"), -2}, {P("132"), -2}, {P("321"), -2}, {P("231"), 1}, {P("312"), 1}};
  const auto F1 = std::vector<std::pair<std::vector<int>, double>>{{P("123"), 2}, {P("213"), -1}};
  const auto F2 = std::vector<std::pair<std::vector<int>, double>>{{P("123"), 2}, {P("132"), -1}};
  auto t = [](int bl, int cpw, int threads, int pad, int variant, int item_tiles) {
    return spinsum_tile_t{bl, cpw, threads, pad, variant, item_tiles};
  };
  std::vector<Case> cases = {
      {"3d 2x32^3", {2, 32, 32, 32}, 1, 3, {A3}, 0, SPINSUM_F64, 1,
       {t(8, 1, 0, 0, 1, 0), t(5, 1, 0, 1, 3, 0), t(12, 1, 0, 1, 2, 0), t(4, 1, 0, 0, 4, 0),
        t(32, 1, 0, 0, 0, 0)}},
      {"3d 96^3 line order", {96, 96, 96}, 0, 3, {A3}, 0, SPINSUM_F64, 0, {t(8, 1, 0, 0, 1, 0)}},
      {"3d fp32 2x24^3 chained", {2, 24, 24, 24}, 1, 3, {F1, F2}, SPINSUM_FLAG_CHAIN_STAGES,
       SPINSUM_F32, 1, {t(8, 1, 0, 0, 1, 0)}},
      {"3d multi-pass", {3, 16, 16, 16}, 1, 3, {F1, F2}, SPINSUM_FLAG_MULTI_PASS, SPINSUM_F64, 0,
       {}},
      {"4d 12^4 random", {1, 12, 12, 12, 12}, 1, 4, {all_perms(4, 7)}, 0, SPINSUM_F64, 1,
       {t(4, 1, 0, 0, 1, 0), t(6, 1, 0, 0, 1, 6), t(3, 1, 0, 1, 3, 0)}},
      {"4d 40^4 line order", {40, 40, 40, 40}, 0, 4, {all_perms(4, 3)}, 0, SPINSUM_F64, 1, {}},
      {"2d 3x40^2", {3, 40, 40}, 1, 2, {{{P("12"), 1}, {P("21"), -1}}}, 0, SPINSUM_F64, 0,
       {t(8, 1, 0, 0, 1, 0)}},
      {"inner run 8", {2, 12, 12, 12, 8}, 1, 3, {A3}, 0, SPINSUM_F64, 1, {t(4, 1, 0, 0, 1, 0)}},
      {"inner runs 3x2", {2, 10, 10, 10, 3, 2}, 1, 3, {A3}, 0, SPINSUM_F32, 0, {}},
      {"index pairs", {2, 3, 3, 3, 8, 8, 8}, 4, 3, {A3}, SPINSUM_FLAG_INDEX_PAIRS, SPINSUM_F64, 1,
       {t(4, 1, 0, 0, 1, 0)}},
      {"index pairs 4d", {2, 2, 2, 2, 3, 3, 3, 3}, 4, 4, {all_perms(4, 5)},
       SPINSUM_FLAG_INDEX_PAIRS, SPINSUM_F64, 0, {}},
      {"subgroup fig1b", {2, 12, 12, 12}, 1, 3, {{{P("123"), 1}, {P("213"), 1}}}, 0, SPINSUM_F64,
       1, {t(4, 1, 0, 0, 1, 0)}},
      {"subgroup 4d axes 1-3", {2, 6, 6, 6, 6}, 1, 4,
       {{{P("1234"), 2}, {P("1243"), -1}}, {{P("1234"), 1}, {P("1342"), 3}}}, 0, SPINSUM_F64, 0,
       {}},
      {"full group flag", {2, 12, 12, 12}, 1, 3, {{{P("123"), 1}, {P("213"), 1}}},
       SPINSUM_FLAG_FULL_GROUP, SPINSUM_F64, 1, {}},
      {"empty", {0, 8, 8, 8}, 1, 3, {A3}, 0, SPINSUM_F64, 1, {}},
  };
  for (const Case& c : cases) run_case(c);
  batched_case("batched trailing", {{3, 4, 4, 4}, {2, 9, 9, 9}, {1, 13, 13, 13}, {4, 6, 6, 6}}, -1,
               3, A3);
  batched_case("batched inner", {{3, 4, 4, 4, 2}, {2, 9, 9, 9, 3}, {1, 17, 17, 17, 1}}, 1, 3, A3);

  // arguments the planner must refuse
  spinsum_plan_t p = nullptr;
  const int64_t sh[] = {2, 4, 4, 4};
  const int bad_perm[] = {0, 0, 1};
  const int one = 1;
  const double a1 = 1.0;
  check(spinsum_plan(&p, 4, sh, 1, 3, 1, &one, bad_perm, &a1, SPINSUM_F64, 0,
                     SPINSUM_FLAG_HOST_ONLY) != SPINSUM_OK && !p,
        "non-bijection refused");
  const int64_t sh2[] = {2, 4, 4, 5};
  const int id3[] = {0, 1, 2};
  check(spinsum_plan(&p, 4, sh2, 1, 3, 1, &one, id3, &a1, SPINSUM_F64, 0,
                     SPINSUM_FLAG_HOST_ONLY) != SPINSUM_OK && !p,
        "unequal extents refused");
  check(spinsum_plan(&p, 4, sh, 1, 5, 1, &one, id3, &a1, SPINSUM_F64, 0,
                     SPINSUM_FLAG_HOST_ONLY) != SPINSUM_OK && !p,
        "d = 5 refused");
  check(spinsum_plan(nullptr, 4, sh, 1, 3, 1, &one, id3, &a1, SPINSUM_F64, 0,
                     SPINSUM_FLAG_HOST_ONLY) != SPINSUM_OK,
        "null plan pointer refused");
  check(spinsum_plan_get_info(nullptr, nullptr) != SPINSUM_OK, "null info refused");
  spinsum_plan_destroy(nullptr);
  std::printf("%s\n", g_fail ? "FAILED" : "PASSED");
  return g_fail ? 1 : 0;
}
