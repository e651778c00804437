"""Host threads the CPU oracle may use in the tests: OMP_NUM_THREADS when
it is set (the process's share of the machine), else every CPU this process
may run on."""
import os


def host_threads() -> int:
    env = os.environ.get("OMP_NUM_THREADS", "").strip()
    if env.isdigit() and int(env) > 0:
        return int(env)
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except (AttributeError, OSError):
        return max(1, os.cpu_count() or 1)


HOST_THREADS = host_threads()
