"""Host logic of the server's device-byte accounting (no GPU): reuse by best
fit, growth charged old+new, release of pooled plans under pressure, waiting
when running requests hold the budget, and conservation of counted bytes."""
import random

from paper_2009_12457_amd.serve import PlanPool, default_p, footprint_estimate


class FakePlan:
    def __init__(self, name):
        self.name = name
        self.destroyed = False

    def destroy(self):
        assert not self.destroyed
        self.destroyed = True


def test_fresh_take_and_settle():
    pool = PlanPool(1000)
    plan, charge = pool.take(400)
    assert plan is None and charge == 400 and pool.in_use == 400
    held = pool.settle(charge, 350)
    assert held == 350 and pool.in_use == 350
    a = FakePlan("a")
    pool.give_back(a, held)
    assert pool.in_use == 350  # a pooled plan still holds its bytes


def test_best_fit_reuse():
    pool = PlanPool(10_000)
    plans = {h: FakePlan(h) for h in (300, 500, 900)}
    for h, p in plans.items():
        pool.in_use += h
        pool.give_back(p, h)
    plan, charge = pool.take(450)
    assert plan is plans[500] and charge == 500
    assert pool.in_use == 1700
    plan, charge = pool.take(100)
    assert plan is plans[300] and charge == 300


def test_growth_charged_old_plus_new_and_others_released_largest_first():
    pool = PlanPool(2000)
    a, b, c = FakePlan("a"), FakePlan("b"), FakePlan("c")
    for p, h in ((a, 600), (b, 300), (c, 200)):
        pool.in_use += h
        pool.give_back(p, h)
    # 1100 held; a request of 1000 fits no pooled plan: the largest (a) grows,
    # and b is released (largest of the others) to bring 1100+1000 under 2000
    plan, charge = pool.take(1000)
    assert plan is a and charge == 1600
    assert b.destroyed and not c.destroyed and not a.destroyed
    assert pool.in_use == 600 + 200 + 1000
    assert pool.in_use <= pool.budget
    pool.settle(charge, 1000)
    assert pool.in_use == 1200


def test_grown_plan_released_when_nothing_else_helps():
    pool = PlanPool(1000)
    a = FakePlan("a")
    pool.in_use += 500
    pool.give_back(a, 500)
    plan, charge = pool.take(800)  # 500 + 800 > 1000: a goes, a fresh plan is made
    assert plan is None and charge == 800 and a.destroyed and pool.in_use == 800


def test_waits_while_running_requests_hold_the_budget():
    pool = PlanPool(1000)
    _, c1 = pool.take(700)
    assert pool.take(400) is None
    pool.drop(None, c1)
    assert pool.in_use == 0
    assert pool.take(400) == (None, 400)


def test_conservation_random_sequences():
    rng = random.Random(7)
    for trial in range(50):
        pool = PlanPool(rng.randint(1000, 5000))
        running = []  # (plan, charge)
        for step in range(200):
            r = rng.random()
            if r < 0.5:
                need = rng.randint(1, pool.budget)
                got = pool.take(need)
                if got is not None:
                    plan, charge = got
                    held = rng.randint(max(1, need // 2), need)
                    if plan is not None:
                        held = max(held, charge - need)  # a reused plan keeps at least its old buffers
                    charge = pool.settle(charge, held)
                    running.append((plan or FakePlan(step), charge))
            elif running:
                plan, charge = running.pop(rng.randrange(len(running)))
                if rng.random() < 0.1:
                    pool.drop(plan, charge)
                else:
                    pool.give_back(plan, charge)
            counted = sum(c for _, c in running) + sum(h for _, h in pool.idle)
            assert pool.in_use == counted
            assert all(not p.destroyed for p, _ in pool.idle)
        pool.clear()
        assert pool.in_use == sum(c for _, c in running)


def test_footprint_estimate_and_p_prior():
    assert default_p(1000, 32000) == 4
    assert default_p(10, 2) == 4 and default_p(3, 4) == 3  # never more parts than vertices
    assert default_p(1 << 20, 2 * (8 << 20)) == 8
    assert default_p(1 << 22, 2 * (64 << 20)) == 16
    # dense graphs: every vertex may store boundaries, and those stay within
    # the out-rows' 4 B per edge, so only the per-edge bytes grow
    a = footprint_estimate(1 << 16, 1 << 22, 16)
    b = footprint_estimate(1 << 16, 1 << 23, 16)
    assert b - a == (42 + 4) * (1 << 21)
    # sparse graphs at large p: stored boundary rows are bounded by nnz/33
    c = footprint_estimate(1 << 20, 1 << 20, 64)
    assert c - footprint_estimate(1 << 20, 1 << 20, 1) <= 4 * 65 * ((1 << 20) // 33) + 64 * 64 * 65 * 66 // 6
