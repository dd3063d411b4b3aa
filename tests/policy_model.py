"""A plain model of the partition cache's slot policy, written from its
specification (the rendered views' missing partitions take an empty slot,
least recently used first, else the least recently used slot the batch does
not need; then the upcoming views' missing partitions take what is left), with
each upload's release batch: the copy into a slot may start only once the
work enqueued before the first batch after the slot's previous use has
finished, and only the last 16 batch start points are kept."""

RING = 16


class Capacity(Exception):
    pass


class PolicyModel:
    def __init__(self, n_parts: int, n_slots: int):
        self.n_parts, self.S = n_parts, n_slots
        self.slot_part = [-1] * n_slots
        self.slot_last = [-1] * n_slots
        self.where = {}
        self.batch = 0

    def step(self, need):
        S, b = self.S, self.batch
        rendered = [k for k in range(self.n_parts) if need[k] == 1]
        if len(rendered) > S:
            raise Capacity(len(rendered))
        hits = [k for k in rendered if k in self.where]
        taken = {self.where[k] for k in hits}
        for k in hits:
            self.slot_last[self.where[k]] = b
        uploads, ev = [], 0

        def victim():
            free = [s for s in range(S) if s not in taken and self.slot_part[s] < 0]
            cand = free or [s for s in range(S) if s not in taken]
            return min(cand, key=lambda s: (self.slot_last[s], s)) if cand else None

        def claim(k, v, ahead):
            nonlocal ev
            prev = self.slot_last[v]
            rel = -1 if prev < 0 else max(prev + 1, b - (RING - 1))
            if self.slot_part[v] >= 0:
                del self.where[self.slot_part[v]]
                ev += 1
            self.slot_part[v], self.slot_last[v], self.where[k] = k, b, v
            taken.add(v)
            uploads.append((k, v, rel, ahead))

        for k in rendered:
            if k not in self.where:
                claim(k, victim(), 0)
        upcoming = [k for k in range(self.n_parts) if need[k] == 2]
        for k in upcoming:
            if k in self.where:
                taken.add(self.where[k])
                self.slot_last[self.where[k]] = b
        pre = 0
        for k in upcoming:
            if k in self.where:
                continue
            v = victim()
            if v is None:
                continue
            claim(k, v, 1)
            pre += 1
        self.batch += 1
        return dict(needed=len(rendered), hits=len(hits), uploads=len(uploads), evictions=ev, prefetched=pre,
                    upload_list=uploads)

    def evict_all(self):
        self.slot_part = [-1] * self.S
        self.where = {}
