// Host check of the LDS layout of the one-task-per-lane Jacobi solves
// (orders up to 12): built from the kernel source itself with the device
// code left out, it walks every entry and every task of each padded order.
#include "../paper_2603_10295_amd/csrc/jacobi.hip"

#include <cstdio>
#include <map>
#include <set>
#include <string>

namespace ephw {
void set_error(const std::string&) {}
}  // namespace ephw

using namespace ephw;

template <int NP>
int check() {
  using L = SmallLayout<NP>;
  constexpr int N2 = L::N2, NT = L::NT, RS = L::RS;
  int bad = 0;
  auto fail = [&](const char* what, int a, int b) {
    if (bad < 10) std::printf("NP %d: %s (%d, %d)\n", NP, what, a, b);
    ++bad;
  };
  // every entry in the data region, one slot each; A below its diagonal
  // shares its transpose's slot (flagged), A and V apart
  std::set<uint32_t> a_slots, v_slots;
  for (int r = 0; r < N2; ++r)
    for (int c = 0; c < N2; ++c) {
      const uint32_t a = entry_offset<NP>(false, r, c), v = entry_offset<NP>(true, r, c);
      if ((a & 0x7fffu) >= L::data_elems || v >= L::data_elems) fail("offset outside the data region", r, c);
      if (((a & 0x8000u) != 0) != (r > c)) fail("conjugate flag", r, c);
      if (r > c && (a & 0x7fffu) != entry_offset<NP>(false, c, r)) fail("transpose slot", r, c);
      if (r <= c && !a_slots.insert(a).second) fail("A slot used twice", r, c);
      if (!v_slots.insert(v).second) fail("V slot used twice", r, c);
    }
  for (uint32_t s : a_slots)
    if (v_slots.count(s)) fail("A and V share a slot", (int)s, 0);
  if (a_slots.size() != (size_t)N2 * (N2 + 1) / 2 || v_slots.size() != (size_t)N2 * N2) fail("slot count", 0, 0);
  // a round: task t loads its entry e from e RS + t (entry 2 of a diagonal
  // block of A is entry 1 conjugated) and stores it to its moved position;
  // the stores cover every slot the next round loads
  std::set<uint32_t> loaded, stored;
  for (int t = 0; t < NT; ++t) {
    bool is_v;
    int i, j;
    decode_task<NP>(t, is_v, i, j);
    const int rr[2] = {i, N2 - 1 - i}, cc[2] = {j, N2 - 1 - j};
    for (int e = 0; e < 4; ++e) {
      const int r = rr[e >> 1], c = cc[e & 1];
      const uint32_t got = entry_offset<NP>(is_v, r, c);
      const bool shared = !is_v && i == j && e == 2;
      const bool below = !is_v && r > c;
      const uint32_t want = (uint32_t)((shared ? 1 : e) * RS + t) | (below ? 0x8000u : 0u);
      if (got != want) fail("load offset of task, entry", t, e);
      loaded.insert(got & 0x7fffu);
      stored.insert(entry_offset<NP>(is_v, is_v ? r : next_pos(r, N2), next_pos(c, N2)) & 0x7fffu);
    }
  }
  if (loaded != stored) fail("stores do not cover the loaded slots", (int)loaded.size(), (int)stored.size());
  // a sweep of N2 - 1 moves brings every position back
  for (int p = 0; p < N2; ++p) {
    int x = p;
    for (int k = 0; k < N2 - 1; ++k) x = next_pos(x, N2);
    if (x != p) fail("position not back after a sweep", p, x);
  }
  std::printf("NP %d: %zu A slots, %zu V slots, %d data slots, %d failures\n", NP, a_slots.size(), v_slots.size(),
              (int)L::data_elems, bad);
  return bad;
}

int main() {
  const int bad = check<1>() + check<2>() + check<3>() + check<4>() + check<5>() + check<6>();
  if (bad == 0) std::printf("jacobi_layout_check: ok\n");
  return bad ? 1 : 0;
}
