import os
import shutil
import subprocess
import sys
import tempfile
import threading
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


import pytest  # noqa: E402


@pytest.fixture(autouse=True)
def _announce_gpu_case(request):
    """Name each GPU test on the real stderr before it touches the device."""
    if request.node.get_closest_marker("gpu") is not None:
        sys.__stderr__.write("\n[gpu case] %s\n" % request.node.nodeid)
        sys.__stderr__.flush()
    yield


class OracleFarm:
    """Full-size oracle runs (tests/oracle_jobs.py) as child processes.

    At most ``slots`` jobs run at once, in the order given; ``wait(job)``
    blocks until a job's file exists (printing progress), and fails with the
    oracle's traceback if the job failed.
    """

    def __init__(self, jobs, slots):
        self.dir = tempfile.mkdtemp(prefix="mgc_oracle_")
        self.pending = list(jobs)
        self.running = {}
        self.failed = {}
        self.slots = slots
        self.lock = threading.Lock()
        self.stop = False
        self.thread = threading.Thread(target=self._loop, daemon=True)
        self.thread.start()

    def _start(self, job):
        env = dict(os.environ)
        env.setdefault("OMP_NUM_THREADS", "2")
        log = open(os.path.join(self.dir, job + ".log"), "w")
        p = subprocess.Popen([sys.executable, "-m", "tests.oracle_jobs", job, self.dir],
                             cwd=ROOT, env=env, stdout=log, stderr=subprocess.STDOUT)
        self.running[job] = (p, log, time.time())
        sys.__stderr__.write("[oracle job] started %s\n" % job)
        sys.__stderr__.flush()

    def _loop(self):
        while not self.stop:
            with self.lock:
                for job, (p, log, t0) in list(self.running.items()):
                    rc = p.poll()
                    if rc is not None:
                        log.close()
                        del self.running[job]
                        if rc != 0:
                            self.failed[job] = rc
                        sys.__stderr__.write("[oracle job] %s finished (rc %d, %.0f s)\n"
                                             % (job, rc, time.time() - t0))
                        sys.__stderr__.flush()
                while self.pending and len(self.running) < self.slots:
                    self._start(self.pending.pop(0))
                if not self.pending and not self.running:
                    return
            time.sleep(0.5)

    def wait(self, job, timeout=1500.0):
        from tests import oracle_jobs
        path = oracle_jobs.output_path(self.dir, job)
        err = os.path.join(self.dir, job + ".err")
        t0 = time.time()
        last = t0
        while not os.path.exists(path):
            if os.path.exists(err) or job in self.failed:
                time.sleep(0.5)
                msg = open(err).read() if os.path.exists(err) else "exit %s" % self.failed.get(job)
                pytest.fail("oracle job %s failed:\n%s" % (job, msg))
            if time.time() - t0 > timeout:
                pytest.fail("oracle job %s did not finish in %.0f s" % (job, timeout))
            if time.time() - last > 20:
                last = time.time()
                sys.__stderr__.write("[oracle job] waiting for %s (%.0f s)\n" % (job, last - t0))
                sys.__stderr__.flush()
            time.sleep(0.5)
        return path

    def close(self):
        self.stop = True
        with self.lock:
            for p, log, _ in self.running.values():
                p.kill()
                p.wait()
                log.close()
            self.running.clear()
        shutil.rmtree(self.dir, ignore_errors=True)


_FARM = {}


def pytest_collection_finish(session):
    """Start the full-size oracle runs when selected GPU tests need them and
    a GPU device node exists (checked without initialising the GPU)."""
    wanted = any("oracle_farm" in getattr(it, "fixturenames", ()) for it in session.items)
    if wanted and os.path.exists("/dev/kfd"):
        from tests import oracle_jobs
        slots = max(1, min(6, (len(os.sched_getaffinity(0)) or 2) // 2))
        _FARM["farm"] = OracleFarm(oracle_jobs.ALL_JOBS, slots)


def pytest_sessionfinish(session, exitstatus):
    farm = _FARM.pop("farm", None)
    if farm is not None:
        farm.close()


@pytest.fixture(scope="session")
def oracle_farm():
    farm = _FARM.get("farm")
    if farm is None:
        pytest.skip("full-size oracle runs were not started (no GPU device node)")
    return farm
