"""CPU test of the queueing model of the request loop (serve_model.py): calibrated to the
saturated rate of the last GPU run of the serving leg (271.6 frames/s on one stream), the
round policy reproduces that run's latency at 0.7 of saturation (p99 60.4 ms measured,
p50 8.2 ms), and the policies keep the structure the design analysis rests on: a budget
of large-frame work per round shortens the small frames' tail and lengthens the 4K frames',
never raises throughput, and the overall p99 stays near the 4K frames' own."""
import numpy as np

import serve_model as SM

MEASURED_SAT_FPS, MEASURED_P50_MS, MEASURED_P99_MS = 271.6, 8.20, 60.4


def test_serve_model_reproduces_the_measured_tail_and_keeps_its_structure():
    R, rows = SM.table(sat_fps=MEASURED_SAT_FPS)
    by = {(pol, b): (sat, p50, p99, per) for pol, b, sat, p50, p99, per in rows}
    sat, p50, p99, per = by[("rounds", None)]
    print(rows)
    assert abs(sat - 1.0) < 1e-3
    assert abs(p99 - MEASURED_P99_MS) <= 0.1 * MEASURED_P99_MS
    assert abs(p50 - MEASURED_P50_MS) <= 0.3 * MEASURED_P50_MS
    small, big = "960x540", "3840x2160"
    budgets = [2.0, 5.0, 10.0, 20.0]
    small_p99 = [by[("budget", b)][3][small] for b in budgets]
    big_p99 = [by[("budget", b)][3][big] for b in budgets]
    assert all(np.diff(small_p99) > 0) and all(np.diff(big_p99) < 0)   # the trade, budget by budget
    assert small_p99[0] < 0.3 * per[small] and big_p99[0] > 1.5 * per[big]
    assert all(by[("budget", b)][0] <= 1.0 for b in budgets)
    assert abs(by[("one_large", None)][0] - 1.0) < 1e-3 and abs(by[("one_oldest", None)][0] - 1.0) < 1e-3
    # small frames first halves their tail whichever large frame goes next
    assert by[("one_large", None)][3][small] < 0.6 * per[small] and by[("one_oldest", None)][3][small] < 0.6 * per[small]
    assert all(r[4] > 0.8 * p99 for r in rows)   # no policy takes the overall p99 far below
