"""CPU check of the error bound behind the stage-1 back-face test of union-box strips: with fast
window positions within 1/32 px of their snapped positions (the fast test's margin), a fast signed
area below minus the bound 2m(|a.x| + |a.y| + |b.x| + |b.y|) + 8m^2 + 2^-20 (|a.x b.y| + |a.y b.x|)
(times 1 + 2^-16, all in binary32 as the kernel evaluates it) always means a negative snapped area
(snapping to 1/256 px as the exact path does), for either winding of the strip order."""
import numpy as np

f32 = np.float32
M = f32(1.0 / 32.0)


def provably_back(p0, p1, p2, even):
    ax, ay = f32(p1[0] - p0[0]), f32(p1[1] - p0[1])
    bx, by = f32(p2[0] - p0[0]), f32(p2[1] - p0[1])
    P, Q = f32(ax * by), f32(ay * bx)
    A = f32(P - Q) if even else f32(Q - P)
    B = f32(f32(f32(2.0) * M) * f32(f32(abs(ax) + abs(ay)) + f32(abs(bx) + abs(by))))
    B = f32(B + f32(f32(8.0) * M * M))
    B = f32(B + f32(f32(1.0 / 1048576.0) * f32(abs(P) + abs(Q))))
    return A < -f32(B * f32(1.0 + 1.0 / 65536.0))


def test_provably_back_facing_means_a_negative_snapped_area():
    rng = np.random.default_rng(7)
    decided = 0
    for _ in range(40000):
        size = 10 ** rng.uniform(-1.5, 1.7)
        exact = rng.uniform(0, 4000, 2) + rng.normal(size=(3, 2)) * size
        X = np.rint(exact * 256.0)
        area = (X[1, 0] - X[0, 0]) * (X[2, 1] - X[0, 1]) - (X[1, 1] - X[0, 1]) * (X[2, 0] - X[0, 0])
        # fast positions: at most 1/32 px from the snapped ones (the kernel's margin), here up to
        # 1/32 - 1/512 px from the exact position plus the snapping
        fast = (exact + rng.uniform(-1, 1, (3, 2)) * (1 / 32 - 1 / 512)).astype(np.float32)
        for even, order in ((True, [0, 1, 2]), (False, [1, 0, 2]), (True, [1, 2, 0]), (False, [0, 2, 1])):
            q = fast[order]
            if provably_back(q[0], q[1], q[2], even):
                decided += 1
                assert area < 0, (exact, fast, order)
    assert decided > 10000        # the test decides most clearly back-facing triangles
