// Optimal binomial checkpointing schedule (host code).
//
// Checkpointing (paper Sec. 1) keeps a few states and recomputes the others
// from the nearest stored one. Reversing l steps (inputs x_0..x_{l-1} needed in
// reverse order) with s slots, the slot of x_0 included, needs at least
// t(l, s) = r l - C(s + r, r - 1) step evaluations, r the least integer with
// C(s + r, s) >= l (Griewank's binomial bound). The schedule below reaches it:
// advance j steps from the base and store, reverse the tail with one slot
// fewer, then the head with all slots, choosing j to minimise
// j + t(l - j, s - 1) + t(j, s).

#include <algorithm>
#include <cstdint>
#include <vector>

#include "plan.h"

namespace wv {

namespace {

// C(n, k) saturated at `cap` (enough to compare against l)
long long binom_cap(long long n, long long k, long long cap)
{
    if (k < 0 || k > n) return 0;
    k = std::min(k, n - k);
    long double r = 1.0L;
    for (long long q = 1; q <= k; ++q) {
        r = r * (long double)(n - k + q) / (long double)q;
        if (r > (long double)cap) return cap + 1;
    }
    return (long long)(r + 0.5L);
}

long long binom_exact(long long n, long long k)
{
    if (k < 0 || k > n) return 0;
    k = std::min(k, n - k);
    __int128 r = 1;
    for (long long q = 1; q <= k; ++q) r = r * (n - k + q) / q;
    return (long long)r;
}

struct Gen {
    std::vector<RevAction> out;
    std::vector<int> free_slots;
    long long fwd = 0;

    void push(int kind, int a, int b) { out.push_back(RevAction{kind, a, b}); }

    int best_split(int l, int s)
    {
        long long best = -1;
        int arg = 1;
        for (int j = 1; j < l; ++j) {
            const long long c = j + revolve_cost(l - j, s - 1) + revolve_cost(j, s);
            if (best < 0 || c < best) {
                best = c;
                arg = j;
            }
        }
        return arg;
    }

    // deliver x_{a+l-1} .. x_a, x_a held in slot_a, s slots usable (slot_a included)
    void rev(int a, int l, int s, int slot_a)
    {
        if (l == 1) {
            push(2, a, slot_a);
            push(3, a, 0);
            return;
        }
        if (s == 1) {
            for (int q = l - 1; q >= 0; --q) {
                push(2, a, slot_a);
                if (q) {
                    push(0, a, q);
                    fwd += q;
                }
                push(3, a + q, 0);
            }
            return;
        }
        const int j = best_split(l, s);
        push(2, a, slot_a);
        push(0, a, j);
        fwd += j;
        const int slot = free_slots.back();
        free_slots.pop_back();
        push(1, a + j, slot);
        rev(a + j, l - j, s - 1, slot);
        free_slots.push_back(slot);
        rev(a, j, s, slot_a);
    }
};

}  // namespace

long long revolve_cost(long long l, int s)
{
    if (l <= 1) return 0;
    if (s <= 1) return l * (l - 1) / 2;
    long long r = 0;
    while (binom_cap(s + r, s, l) < l) ++r;
    return r * l - (r >= 1 ? binom_exact(s + r, r - 1) : 0);
}

std::vector<RevAction> revolve_schedule(int nsteps, int nslots, long long* forward_steps)
{
    if (nsteps < 1 || nslots < 1) throw Error{WV_EINVAL, "revolve: nsteps and nslots must be >= 1"};
    Gen g;
    for (int q = nslots - 1; q >= 1; --q) g.free_slots.push_back(q);
    g.rev(0, nsteps, nslots, 0);
    if (forward_steps) *forward_steps = g.fwd;
    return g.out;
}

std::vector<int> sweep_snapshots(const std::vector<RevAction>& acts, int T, size_t* first_deliver)
{
    std::vector<int> snap(T + 1, 0);
    size_t q = 0;
    for (; q < acts.size(); ++q) {
        if (acts[q].kind == 3) break;
        if (acts[q].kind == 1) {
            WV_REQUIRE(acts[q].a >= 0 && acts[q].a <= T, WV_EINVAL, "sweep_snapshots: store outside the solve");
            snap[acts[q].a] = acts[q].b;
        }
    }
    *first_deliver = q;
    return snap;
}

}  // namespace wv
